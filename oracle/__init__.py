"""CPU oracle for the Larger-than-Life step (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg use this
package. It shares no code with the HIP library and never imports it.

Two independent implementations of the same definition:

* ``count`` / ``step`` / ``run``: the C oracle in ``ltl_oracle.c`` (direct
  (2r+1)^2 box count with a dead ghost halo or on a torus, then the LTL
  transition), OpenMP over rows, reached through ctypes;
* ``np_count`` / ``np_step`` / ``np_run``: a NumPy transcription for tiny grids
  (zero-padded shifted-window sum, or a sum of ``np.roll`` shifts on a torus),
  used to cross-check the C code.

Paper passages followed: "Formulation of CAT", Eq. 2-3 (the Moore reduction is a
box sum of half-width r, dead ghost halo; the experiments' periodic boundary, "Experimental design"), the centre remark after Fig. 3
(centre removal when the rule excludes it), the rule notation of "Chosen CA
tests" (R, C, M, S, B, N), and the ping-pong step of "Pseudocode of CAT's
Kernel" (synchronous update). Readings for what the paper leaves open are in the
C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ltl_oracle.c")
_LIB = os.path.join(_HERE, "libltl_oracle.so")
_lib: Optional[ctypes.CDLL] = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP). -march=x86-64-v3 (AVX2) runs on every host
    this is used on and lets gcc vectorize the box sum; the code itself is unchanged."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def use_native() -> str:
    """Compile the same source with -march=native for the host this runs on (into a temporary
    directory) and use that build from here on; the CPU-baseline timing uses it. The code is
    unchanged; only the compiler's instruction selection differs."""
    global _lib
    import tempfile

    out = os.path.join(tempfile.mkdtemp(prefix="ltl_oracle_"), "libltl_oracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-o", out, _SRC])
    _lib = None
    _load(out)
    return out


def _load(path: Optional[str] = None) -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64, I = ctypes.c_int64, ctypes.c_int
        lib.oracle_count.argtypes = [P, I64, I64, I, P]
        lib.oracle_count.restype = None
        lib.oracle_count_periodic.argtypes = [P, I64, I64, I, P]
        lib.oracle_count_periodic.restype = None
        lib.oracle_step_b.argtypes = [P, P, I64, I64, I, I, I, I, I, I, I, I]
        lib.oracle_step_b.restype = I
        lib.oracle_run_b.argtypes = [P, I64, I64, I, I, I, I, I, I, I, I, I]
        lib.oracle_run_b.restype = I
        lib.oracle_count_cross.argtypes = [P, I64, I64, I, I, P]
        lib.oracle_count_cross.restype = None
        lib.oracle_step_nb.argtypes = [P, P, I64, I64, I, I, I, I, I, I, I, I, I]
        lib.oracle_step_nb.restype = I
        lib.oracle_run_nb.argtypes = [P, I64, I64, I, I, I, I, I, I, I, I, I, I]
        lib.oracle_run_nb.restype = I
        lib.oracle_step.argtypes = [P, P, I64, I64, I, I, I, I, I, I, I]
        lib.oracle_step.restype = I
        lib.oracle_run.argtypes = [P, I64, I64, I, I, I, I, I, I, I, I]
        lib.oracle_run.restype = I
        lib.oracle_set_threads.argtypes = [I]
        lib.oracle_set_threads.restype = I
        _lib = lib
    return _lib


def _rule_args(rule):
    R, C, M, S1, S2, B1, B2 = rule.as_tuple() if hasattr(rule, "as_tuple") else rule[:7]
    return int(R), int(C), int(M), int(S1), int(S2), int(B1), int(B2)


def _is_cross(rule) -> bool:
    """Rule code N_N: the paper's simplified Von Neumann neighbourhood (the cross of Eq. 4)."""
    n = getattr(rule, "N", None)
    if n is None and not hasattr(rule, "as_tuple") and len(rule) > 7:
        n = rule[7]
    return n in ("N", ord("N"))


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (n > 0); returns the count in use."""
    return _load().oracle_set_threads(int(n))


def count(grid: np.ndarray, r: int, periodic: bool = False, cross: bool = False) -> np.ndarray:
    """Box count (or, with ``cross``, the count over the plus sign of arm r) of alive
    (== 1) cells, centre included once; dead outside, or on a torus when ``periodic``."""
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    H, W = g.shape
    out = np.empty((H, W), dtype=np.int32)
    if cross:
        _load().oracle_count_cross(g.ctypes.data, H, W, int(r), int(bool(periodic)), out.ctypes.data)
        return out
    fn = _load().oracle_count_periodic if periodic else _load().oracle_count
    fn(g.ctypes.data, H, W, int(r), out.ctypes.data)
    return out


def step(grid: np.ndarray, rule, periodic: bool = False) -> np.ndarray:
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    out = np.empty_like(g)
    rc = _load().oracle_step_nb(g.ctypes.data, out.ctypes.data, g.shape[0], g.shape[1], *_rule_args(rule),
                                int(bool(periodic)), int(_is_cross(rule)))
    if rc != 0:
        raise RuntimeError("oracle_step failed")
    return out


def run(grid: np.ndarray, rule, steps: int, periodic: bool = False) -> np.ndarray:
    g = np.array(grid, dtype=np.uint8, order="C", copy=True)
    rc = _load().oracle_run_nb(g.ctypes.data, g.shape[0], g.shape[1], *_rule_args(rule), int(steps),
                               int(bool(periodic)), int(_is_cross(rule)))
    if rc != 0:
        raise RuntimeError("oracle_run failed")
    return g


# --------------------------------------------------------------- NumPy version
def np_count(grid: np.ndarray, r: int, periodic: bool = False, cross: bool = False) -> np.ndarray:
    """Same count as :func:`count`, as a sum of shifted windows of a zero-padded alive map,
    or of cyclic shifts (``np.roll``) on a torus: (2r+1)^2 offsets for the box, the 4r+1
    offsets of the plus sign for the cross."""
    a = (np.asarray(grid) == 1).astype(np.int32)
    H, W = a.shape
    if cross:
        offs = [(0, d) for d in range(-r, r + 1)] + [(d, 0) for d in range(-r, r + 1) if d != 0]
        out = np.zeros((H, W), dtype=np.int32)
        if periodic:
            for di, dj in offs:
                out += np.roll(a, (-di, -dj), axis=(0, 1))
            return out
        p = np.zeros((H + 2 * r, W + 2 * r), dtype=np.int32)
        p[r:r + H, r:r + W] = a
        for di, dj in offs:
            out += p[r + di:r + di + H, r + dj:r + dj + W]
        return out
    if periodic:
        out = np.zeros((H, W), dtype=np.int32)
        for di in range(-r, r + 1):
            for dj in range(-r, r + 1):
                out += np.roll(a, (-di, -dj), axis=(0, 1))
        return out
    p = np.zeros((H + 2 * r, W + 2 * r), dtype=np.int32)
    p[r:r + H, r:r + W] = a
    out = np.zeros((H, W), dtype=np.int32)
    for di in range(2 * r + 1):
        for dj in range(2 * r + 1):
            out += p[di:di + H, dj:dj + W]
    return out


def np_step(grid: np.ndarray, rule, periodic: bool = False) -> np.ndarray:
    R, C, M, S1, S2, B1, B2 = _rule_args(rule)
    s = np.asarray(grid, dtype=np.int32)
    states = C if C >= 3 else 2
    n = np_count(s, R, periodic, _is_cross(rule))
    c = n - ((s == 1) & (M == 0)).astype(np.int32)
    born = (B1 <= c) & (c <= B2)
    keep = (S1 <= c) & (c <= S2)
    nxt = np.where(s == 0, born.astype(np.int32),
                   np.where(s == 1, np.where(keep, 1, 2 if states > 2 else 0),
                            np.where(s + 1 < states, s + 1, 0)))
    return nxt.astype(np.uint8)


def np_run(grid: np.ndarray, rule, steps: int, periodic: bool = False) -> np.ndarray:
    g = np.asarray(grid, dtype=np.uint8)
    for _ in range(steps):
        g = np_step(g, rule, periodic)
    return g


def cone_run(full_grid_fn, H: int, W: int, rule, steps: int, i: int, j: int,
             radius: int = 0) -> np.ndarray:
    """States after ``steps`` steps of the cells within ``radius`` of (i, j) of an
    H x W grid, computed on the dependency cone only.

    ``full_grid_fn(rows, cols)`` must return the initial states of the window
    ``rows x cols`` (half-open ranges). A cell after k steps depends on the initial
    cells within k*r of it, so the window is that cone clipped to the grid; where
    the clip is the real grid edge the dead halo is exact, and cells near an
    interior cut are not read back.
    """
    R = _rule_args(rule)[0]
    reach = steps * R + radius
    r0, r1 = max(0, i - reach), min(H, i + reach + 1)
    c0, c1 = max(0, j - reach), min(W, j + reach + 1)
    sub = full_grid_fn((r0, r1), (c0, c1))
    res = run(sub, rule, steps)
    a0, a1 = max(0, i - radius), min(H, i + radius + 1)
    b0, b1 = max(0, j - radius), min(W, j + radius + 1)
    return res[a0 - r0:a1 - r0, b0 - c0:b1 - c0]
