"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the Larger-than-Life step. It defines:

* the LTL rule record ``Rule`` (notation of the paper's experimental section,
  "Chosen CA tests": ``R_r C_c M_m S_{s1..s2} B_{b1..b2} N_n``) and a parser for
  its text form;
* a counter-based Bernoulli grid generator built on the SplitMix64 output
  function (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): cell ``k = i*W + j`` of a grid with seed ``s`` takes
  the ``k``-th output of the SplitMix64 stream started at state ``s`` and is alive
  iff the high 32 bits are below ``round(p * 2**32)``;
* the benchmark workloads (Life 256^2, Bosco-type R5 4096^2, the radius sweep
  on 16384^2, the 512-instance batch and the 8-state decay rule on 32768^2),
  which stand in for the paper's random LTL grids ("Experimental Design":
  uniform random initial states of density delta).

The paper runs periodic boundaries; the workloads here use a dead ghost halo.
"""
from __future__ import annotations

import dataclasses
import json
import math
import re
from typing import List, Optional, Sequence, Tuple

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1


# --------------------------------------------------------------------------- rules
@dataclasses.dataclass(frozen=True)
class Rule:
    """One LTL rule ``R_r C_c M_m S_{s1..s2} B_{b1..b2} N_n``.

    ``C`` is the number of states (0 and 2 both mean two states), ``M`` says
    whether the centre cell is part of its own neighbourhood, the S and B ranges
    are inclusive, and ``N`` is ``'M'`` (Moore) or ``'N'`` (Von Neumann).
    """

    R: int
    C: int
    M: int
    S1: int
    S2: int
    B1: int
    B2: int
    N: str = "M"

    def text(self) -> str:
        return f"R{self.R},C{self.C},M{self.M},S{self.S1}..{self.S2},B{self.B1}..{self.B2},N{self.N}"

    def as_tuple(self) -> Tuple[int, int, int, int, int, int, int]:
        return (self.R, self.C, self.M, self.S1, self.S2, self.B1, self.B2)


_RULE_RE = re.compile(
    r"^\s*R(?P<R>\d+)\s*,?\s*C(?P<C>\d+)\s*,?\s*M(?P<M>\d+)\s*,?\s*"
    r"S(?P<S1>\d+)\.\.(?P<S2>\d+)\s*,?\s*B(?P<B1>\d+)\.\.(?P<B2>\d+)\s*,?\s*N_?(?P<N>[MN])\s*$"
)


def parse_rule(text: str) -> Rule:
    """Parse ``"R5,C0,M1,S34..58,B34..45,NM"`` (commas and spaces optional)."""
    m = _RULE_RE.match(text.replace(" ", ""))
    if m is None:
        raise ValueError(f"not an LTL rule: {text!r}")
    g = m.groupdict()
    return Rule(int(g["R"]), int(g["C"]), int(g["M"]), int(g["S1"]), int(g["S2"]),
                int(g["B1"]), int(g["B2"]), g["N"])


LIFE = Rule(1, 0, 1, 3, 4, 3, 3)          # Game of Life with the centre counted
BOSCO_M1 = Rule(5, 0, 1, 34, 58, 34, 45)  # Bosco-type rule on the 4096^2 workload
DECAY_C8 = Rule(16, 8, 0, 300, 500, 330, 420)


# ----------------------------------------------------------------- SplitMix64
def _mix_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= np.uint64(MIX1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(MIX2)
    z ^= z >> np.uint64(31)
    return z


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """k-th output (k >= 0) of the SplitMix64 stream with initial state ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (k + np.uint64(1)) * np.uint64(GAMMA)
        return _mix_np(z)


def splitmix64_scalar(seed: int, k: int) -> int:
    z = (seed + (k + 1) * GAMMA) & _M64
    z = ((z ^ (z >> 30)) * MIX1) & _M64
    z = ((z ^ (z >> 27)) * MIX2) & _M64
    return z ^ (z >> 31)


def threshold32(p: float) -> int:
    """Integer threshold: a draw is a success iff its high 32 bits are below this."""
    if not 0.0 <= p <= 1.0:
        raise ValueError("p must be in [0, 1]")
    return int(round(p * 2.0 ** 32))


def bernoulli_grid(H: int, W: int, p: float, seed: int,
                   rows: Optional[Tuple[int, int]] = None,
                   cols: Optional[Tuple[int, int]] = None) -> np.ndarray:
    """uint8 grid of 0/1 cells, or the sub-window ``rows x cols`` of it."""
    r0, r1 = rows if rows is not None else (0, H)
    c0, c1 = cols if cols is not None else (0, W)
    if not (0 <= r0 <= r1 <= H and 0 <= c0 <= c1 <= W):
        raise ValueError("window outside the grid")
    thr = np.uint64(threshold32(p))
    out = np.empty((r1 - r0, c1 - c0), dtype=np.uint8)
    jj = np.arange(c0, c1, dtype=np.uint64)
    step = max(1, (1 << 22) // max(1, c1 - c0))
    for a in range(r0, r1, step):
        b = min(r1, a + step)
        ii = np.arange(a, b, dtype=np.uint64)[:, None]
        k = ii * np.uint64(W) + jj[None, :]
        u = splitmix64(seed, k)
        out[a - r0:b - r0] = ((u >> np.uint64(32)) < thr).astype(np.uint8)
    return out


def bernoulli_grid_torch(H: int, W: int, p: float, seed: int, device="cpu"):
    """Same cells as :func:`bernoulli_grid`, generated with torch int64 ops on ``device``.

    Used to build large grids directly in device memory. int64 products wrap
    modulo 2**64 and right shifts are made logical by masking.
    """
    import torch

    def s64(x: int) -> int:
        x &= _M64
        return x - (1 << 64) if x >= (1 << 63) else x

    def lshr(z, n):
        return (z >> n) & ((1 << (64 - n)) - 1)

    thr = threshold32(p)
    out = torch.empty((H, W), dtype=torch.uint8, device=device)
    step = max(1, (1 << 24) // max(1, W))
    jj = torch.arange(W, dtype=torch.int64, device=device)
    for a in range(0, H, step):
        b = min(H, a + step)
        ii = torch.arange(a, b, dtype=torch.int64, device=device)[:, None]
        k = ii * W + jj[None, :]
        z = (k + 1) * s64(GAMMA) + s64(seed)
        z = (z ^ lshr(z, 30)) * s64(MIX1)
        z = (z ^ lshr(z, 27)) * s64(MIX2)
        z = z ^ lshr(z, 31)
        out[a:b] = (lshr(z, 32) < thr).to(torch.uint8)
    return out


def state_grid(H: int, W: int, C: int, seed: int) -> np.ndarray:
    """Uniform random states in [0, max(C, 2)) from the same counter stream (tests only)."""
    n = max(C, 2)
    k = np.arange(H * W, dtype=np.uint64)
    u = splitmix64(seed, k) >> np.uint64(32)
    return ((u * np.uint64(n)) >> np.uint64(32)).astype(np.uint8).reshape(H, W)


# ------------------------------------------------------------------ workloads
def sweep_rule(r: int) -> Rule:
    """Radius-sweep rule: S = [0.25, 0.45] x N and B = [0.27, 0.34] x N, N = (2r+1)^2, floored."""
    n = (2 * r + 1) ** 2
    return Rule(r, 0, 1, (25 * n) // 100, (45 * n) // 100, (27 * n) // 100, (34 * n) // 100)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    H: int
    W: int
    rule: Rule
    steps: int
    seed: int
    p: float = 0.5


WORKLOADS = {
    "life256": Workload("life256", 256, 256, LIFE, 64, 1),
    "bosco4096": Workload("bosco4096", 4096, 4096, BOSCO_M1, 100, 2),
    "decay32768": Workload("decay32768", 32768, 32768, DECAY_C8, 20, 5),
}


def sweep_workload(r: int, side: int = 16384, steps: int = 50) -> Workload:
    return Workload(f"sweep{side}_r{r}", side, side, sweep_rule(r), steps, 3)


@dataclasses.dataclass(frozen=True)
class Instance:
    H: int
    W: int
    rule: Rule
    seed: int


def batch_instances(count: int = 512, seed: int = 4, side_lo: int = 128,
                    side_hi: int = 2048, max_r: int = 16) -> List[Instance]:
    """The batched workload: square sides log-uniform in [side_lo, side_hi], r uniform in
    1..max_r, S and B each a sorted pair of integers drawn uniformly from
    [ceil(0.2 N), floor(0.5 N)], N = (2r+1)^2; M1, two states, Moore.
    Grid seed of instance i is the i-th SplitMix64 output of the stream ``seed``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        side = min(max(side, side_lo), side_hi)
        r = int(rng.integers(1, max_r + 1))
        n = (2 * r + 1) ** 2
        lo, hi = math.ceil(0.2 * n), math.floor(0.5 * n)
        s = sorted(int(x) for x in rng.integers(lo, hi + 1, size=2))
        b = sorted(int(x) for x in rng.integers(lo, hi + 1, size=2))
        gseed = splitmix64_scalar(seed, i)
        out.append(Instance(side, side, Rule(r, 0, 1, s[0], s[1], b[0], b[1]), gseed))
    return out


def instances_to_json(insts: Sequence[Instance]) -> str:
    return json.dumps([{"H": x.H, "W": x.W, "rule": x.rule.text(), "seed": x.seed} for x in insts])
