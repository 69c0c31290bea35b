"""ctypes binding of ``libltl.so`` (declared in ``include/ltl.h``).

Functions keep the C names and only marshal arguments; every step of the automaton
runs in the library's HIP kernels. PyTorch supplies device memory and streams.
There is no fallback: if the library is missing or fails to load, the call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libltl.so")

LTL_OK = 0
LTL_ERR_ARG = -1
LTL_ERR_RULE = -2
LTL_ERR_UNSUPPORTED = -3
LTL_ERR_INEXACT = -4
LTL_ERR_SIZE = -5
LTL_ERR_HIP = -6
LTL_ERR_STATE = -7

LTL_CAT_I8 = 0
LTL_CAT_F16 = 1
LTL_CAT_F8 = 2
LTL_DIRECT = 3
METHODS = {"cat_i8": LTL_CAT_I8, "cat_f16": LTL_CAT_F16, "cat_f8": LTL_CAT_F8, "direct": LTL_DIRECT}
LTL_BOUNDARY_DEAD = 0
LTL_BOUNDARY_PERIODIC = 1
BOUNDARIES = {"dead": LTL_BOUNDARY_DEAD, "periodic": LTL_BOUNDARY_PERIODIC}

# every symbol the header declares
EXPORTS = [
    "ltl_buffer_bytes", "ltl_pitch", "ltl_create", "ltl_step", "ltl_read", "ltl_current",
    "ltl_get_tuning", "ltl_set_tuning", "ltl_autotune", "ltl_set_boundary", "ltl_destroy", "ltl_last_error", "ltl_last_error_code",
    "ltl_batch_buffer_bytes", "ltl_batch_create", "ltl_batch_step", "ltl_batch_read",
    "ltl_batch_current", "ltl_batch_get_tuning", "ltl_batch_set_tuning", "ltl_batch_autotune",
    "ltl_batch_destroy", "ltl_tuning_lookup", "ltl_tuning_store", "ltl_run_noalloc",
]


class ltl_rule_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("R", "C", "M", "S1", "S2", "B1", "B2", "N")]


class ltl_tuning_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("steps_per_launch", "tile_rows", "tile_cols", "waves", "use_graph",
                                                   "persistent", "lds_pad")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class LtlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ltl error {code}: {msg}")
        self.code = code


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2406_17284_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    PSZ = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "ltl_buffer_bytes": ([I32, I32, I32, I32], SZ),
        "ltl_pitch": ([I32, ctypes.POINTER(ctypes.c_int32)], I32),
        "ltl_create": ([ctypes.POINTER(P), I32, I32, ctypes.POINTER(ltl_rule_t), I32, P, P, SZ, P, SZ, P], I32),
        "ltl_step": ([P, I32], I32),
        "ltl_read": ([P, P, SZ], I32),
        "ltl_current": ([P, ctypes.POINTER(P), PSZ, ctypes.POINTER(ctypes.c_int64)], I32),
        "ltl_get_tuning": ([P, ctypes.POINTER(ltl_tuning_t)], I32),
        "ltl_set_tuning": ([P, ctypes.POINTER(ltl_tuning_t)], I32),
        "ltl_autotune": ([P, I32, P, SZ, ctypes.POINTER(ltl_tuning_t)], I32),
        "ltl_set_boundary": ([P, I32], I32),
        "ltl_destroy": ([P], I32),
        "ltl_last_error": ([], ctypes.c_char_p),
        "ltl_last_error_code": ([], I32),
        "ltl_batch_buffer_bytes": ([I32, P, P], SZ),
        "ltl_batch_create": ([ctypes.POINTER(P), I32, P, P, P, I32, P, P, SZ, P, P, P], I32),
        "ltl_batch_step": ([P, I32], I32),
        "ltl_batch_read": ([P, I32, P, SZ], I32),
        "ltl_batch_current": ([P, I32, ctypes.POINTER(P), PSZ, ctypes.POINTER(ctypes.c_int64)], I32),
        "ltl_batch_get_tuning": ([P, ctypes.POINTER(ltl_tuning_t)], I32),
        "ltl_batch_set_tuning": ([P, ctypes.POINTER(ltl_tuning_t)], I32),
        "ltl_batch_autotune": ([P, I32, P, SZ, ctypes.POINTER(ltl_tuning_t)], I32),
        "ltl_batch_destroy": ([P], I32),
        "ltl_tuning_lookup": ([I32, I32, ctypes.POINTER(ltl_rule_t), I32, I32, I32, ctypes.POINTER(ltl_tuning_t),
                               ctypes.POINTER(ctypes.c_int32)], I32),
        "ltl_tuning_store": ([I32, I32, ctypes.POINTER(ltl_rule_t), I32, I32, I32, ctypes.POINTER(ltl_tuning_t),
                              ctypes.c_double], I32),
        "ltl_run_noalloc": ([I32, I32, ctypes.POINTER(ltl_rule_t), I32, I32, P, P, SZ, P, SZ, I32, P, SZ, P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def last_error() -> str:
    return load().ltl_last_error().decode()


def _check(rc: int) -> int:
    if rc != LTL_OK:
        raise LtlError(rc, last_error())
    return rc


def _check_size(n: int) -> int:
    """Size-returning calls give 0 on an invalid argument (code and message of the refusal in
    ltl_last_error_code / ltl_last_error)."""
    if n == 0:
        raise LtlError(load().ltl_last_error_code(), last_error())
    return n


def make_rule(rule) -> ltl_rule_t:
    """ltl_rule_t from an ``inputs.Rule`` or a (R, C, M, S1, S2, B1, B2[, N]) tuple."""
    if hasattr(rule, "as_tuple"):
        vals = list(rule.as_tuple()) + [ord(rule.N)]
    else:
        vals = list(rule)
        if len(vals) == 7:
            vals.append(ord("M"))
        elif isinstance(vals[7], str):
            vals[7] = ord(vals[7])
    return ltl_rule_t(*[int(v) for v in vals])


def _stream_handle(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ----------------------------------------------------------------- C-named calls
def ltl_buffer_bytes(H: int, W: int, R: int, method: int) -> int:
    return _check_size(load().ltl_buffer_bytes(int(H), int(W), int(R), int(method)))


def ltl_pitch(W: int) -> int:
    out = ctypes.c_int32(0)
    _check(load().ltl_pitch(W, ctypes.byref(out)))
    return out.value


def ltl_create(H: int, W: int, rule, method: int, buf_a: int, buf_b: int, buf_bytes: int,
               init: int, init_pitch: int, stream=None) -> int:
    h = ctypes.c_void_p(0)
    r = make_rule(rule)
    _check(load().ltl_create(ctypes.byref(h), H, W, ctypes.byref(r), int(method), ctypes.c_void_p(buf_a),
                             ctypes.c_void_p(buf_b), buf_bytes, ctypes.c_void_p(init), init_pitch,
                             ctypes.c_void_p(_stream_handle(stream))))
    return h.value


def ltl_run_noalloc(H: int, W: int, rule, method: int, boundary: int, buf_a: int, buf_b: int, buf_bytes: int,
                    init: int, init_pitch: int, n_steps: int, dst: int, dst_pitch: int, stream=None) -> None:
    r = make_rule(rule)
    _check(load().ltl_run_noalloc(int(H), int(W), ctypes.byref(r), int(method), int(boundary), ctypes.c_void_p(buf_a),
                                  ctypes.c_void_p(buf_b), int(buf_bytes), ctypes.c_void_p(init), int(init_pitch),
                                  int(n_steps), ctypes.c_void_p(dst), int(dst_pitch),
                                  ctypes.c_void_p(_stream_handle(stream))))


def ltl_step(sim: int, n_steps: int) -> None:
    _check(load().ltl_step(ctypes.c_void_p(sim), int(n_steps)))


def ltl_read(sim: int, dst: int, dst_pitch: int) -> None:
    _check(load().ltl_read(ctypes.c_void_p(sim), ctypes.c_void_p(dst), dst_pitch))


def ltl_current(sim: int):
    buf = ctypes.c_void_p(0)
    pitch = ctypes.c_size_t(0)
    steps = ctypes.c_int64(0)
    _check(load().ltl_current(ctypes.c_void_p(sim), ctypes.byref(buf), ctypes.byref(pitch), ctypes.byref(steps)))
    return buf.value, pitch.value, steps.value


def ltl_get_tuning(sim: int) -> ltl_tuning_t:
    t = ltl_tuning_t()
    _check(load().ltl_get_tuning(ctypes.c_void_p(sim), ctypes.byref(t)))
    return t


def ltl_set_tuning(sim: int, steps_per_launch=0, tile_rows=0, tile_cols=0, waves=0, use_graph=1,
                   persistent=0, lds_pad=0) -> None:
    t = ltl_tuning_t(steps_per_launch, tile_rows, tile_cols, waves, use_graph, persistent, lds_pad)
    _check(load().ltl_set_tuning(ctypes.c_void_p(sim), ctypes.byref(t)))


def ltl_autotune(sim: int, probe_steps: int, scratch: int, scratch_bytes: int) -> ltl_tuning_t:
    t = ltl_tuning_t()
    _check(load().ltl_autotune(ctypes.c_void_p(sim), int(probe_steps), ctypes.c_void_p(scratch), int(scratch_bytes),
                               ctypes.byref(t)))
    return t


def ltl_set_boundary(sim: int, boundary: int) -> None:
    _check(load().ltl_set_boundary(ctypes.c_void_p(sim), int(boundary)))


def ltl_destroy(sim: int) -> None:
    _check(load().ltl_destroy(ctypes.c_void_p(sim)))


def ltl_batch_buffer_bytes(H: Sequence[int], W: Sequence[int]) -> int:
    n = len(H)
    ha = (ctypes.c_int32 * n)(*H)
    wa = (ctypes.c_int32 * n)(*W)
    return _check_size(load().ltl_batch_buffer_bytes(n, ha, wa))


def ltl_batch_create(H: Sequence[int], W: Sequence[int], rules, method: int, arena_a: int, arena_b: int,
                     nbytes: int, inits: Sequence[int], init_pitches: Sequence[int], stream=None) -> int:
    n = len(H)
    ha = (ctypes.c_int32 * n)(*H)
    wa = (ctypes.c_int32 * n)(*W)
    ra = (ltl_rule_t * n)(*[make_rule(r) for r in rules])
    ia = (ctypes.c_void_p * n)(*inits)
    pa = (ctypes.c_size_t * n)(*init_pitches)
    h = ctypes.c_void_p(0)
    _check(load().ltl_batch_create(ctypes.byref(h), n, ha, wa, ra, int(method), ctypes.c_void_p(arena_a),
                                   ctypes.c_void_p(arena_b), nbytes, ia, pa,
                                   ctypes.c_void_p(_stream_handle(stream))))
    return h.value


def ltl_batch_step(batch: int, n_steps: int) -> None:
    _check(load().ltl_batch_step(ctypes.c_void_p(batch), int(n_steps)))


def ltl_batch_read(batch: int, index: int, dst: int, dst_pitch: int) -> None:
    _check(load().ltl_batch_read(ctypes.c_void_p(batch), int(index), ctypes.c_void_p(dst), dst_pitch))


def ltl_batch_current(batch: int, index: int):
    buf = ctypes.c_void_p(0)
    pitch = ctypes.c_size_t(0)
    steps = ctypes.c_int64(0)
    _check(load().ltl_batch_current(ctypes.c_void_p(batch), int(index), ctypes.byref(buf), ctypes.byref(pitch),
                                    ctypes.byref(steps)))
    return buf.value, pitch.value, steps.value


def ltl_batch_get_tuning(batch: int) -> ltl_tuning_t:
    t = ltl_tuning_t()
    _check(load().ltl_batch_get_tuning(ctypes.c_void_p(batch), ctypes.byref(t)))
    return t


def ltl_batch_set_tuning(batch: int, steps_per_launch=0, tile_rows=0, tile_cols=0, waves=0, use_graph=1,
                         persistent=0, lds_pad=0) -> None:
    t = ltl_tuning_t(steps_per_launch, tile_rows, tile_cols, waves, use_graph, persistent, lds_pad)
    _check(load().ltl_batch_set_tuning(ctypes.c_void_p(batch), ctypes.byref(t)))


def ltl_batch_autotune(batch: int, probe_steps: int, scratch: int, scratch_bytes: int) -> ltl_tuning_t:
    t = ltl_tuning_t()
    _check(load().ltl_batch_autotune(ctypes.c_void_p(batch), int(probe_steps), ctypes.c_void_p(scratch),
                                     int(scratch_bytes), ctypes.byref(t)))
    return t


def ltl_batch_destroy(batch: int) -> None:
    _check(load().ltl_batch_destroy(ctypes.c_void_p(batch)))


def ltl_tuning_lookup(H: int, W: int, rule, method: int, boundary: int = LTL_BOUNDARY_DEAD, batched: int = 0):
    """(tuning, exact) from the tuning table, or None when no entry of the class exists."""
    t = ltl_tuning_t()
    exact = ctypes.c_int32(0)
    r = make_rule(rule)
    rc = load().ltl_tuning_lookup(int(H), int(W), ctypes.byref(r), int(method), int(boundary), int(batched),
                                  ctypes.byref(t), ctypes.byref(exact))
    if rc == LTL_ERR_ARG and "no tuning table entry" in last_error():
        return None
    _check(rc)
    return t, bool(exact.value)


def ltl_tuning_store(H: int, W: int, rule, method: int, boundary: int, batched: int, tuning: dict,
                     ms_per_step: float) -> None:
    t = ltl_tuning_t(*[int(tuning.get(n, 0)) for n, _ in ltl_tuning_t._fields_])
    r = make_rule(rule)
    _check(load().ltl_tuning_store(int(H), int(W), ctypes.byref(r), int(method), int(boundary), int(batched),
                                   ctypes.byref(t), float(ms_per_step)))


# ------------------------------------------------------------ torch-owned memory
def _torch_stream(stream, device):
    """The stream the library enqueues on, as a torch stream (default: the current one)."""
    import torch

    if stream is None:
        return torch.cuda.current_stream(device)
    if isinstance(stream, int):
        return torch.cuda.ExternalStream(stream, device=device)
    return stream


def _join_current(stream, device, tensors) -> None:
    """Order `stream` after torch's current stream (where `tensors` were made or written) and
    keep their memory alive until the work `stream` has queued on them is done."""
    import torch

    cur = torch.cuda.current_stream(device)
    if stream.cuda_stream != cur.cuda_stream:
        stream.wait_stream(cur)
        for t in tensors:
            t.record_stream(stream)


def _current_after(stream, device) -> None:
    """Order torch's current stream after the work queued on `stream` (a read's copy), so torch
    ops on the result see it complete."""
    import torch

    cur = torch.cuda.current_stream(device)
    if stream.cuda_stream != cur.cuda_stream:
        cur.wait_stream(stream)


def _check_out(out, H: int, W: int, device) -> None:
    import torch

    if (out.device != device or out.dtype != torch.uint8 or tuple(out.shape) != (H, W) or out.stride(1) != 1
            or (H > 1 and out.stride(0) < W)):
        raise ValueError(f"out must be a uint8 tensor of shape ({H}, {W}) on {device} with rows of unit "
                         "column stride that do not overlap")


class Simulation:
    """One automaton whose two ping-pong buffers are torch uint8 tensors on the GPU.

    init      2-D uint8 CUDA tensor of states (each < max(C, 2)); copied at creation.
    rule      an ``inputs.Rule`` or anything with R, C, M, S1, S2, B1, B2 (and N) attributes.
    method    "cat_i8" | "cat_f16" | "cat_f8" | "direct" (or the ltl_method_t value).
    stream    torch stream (or raw HIP stream handle) the library enqueues on (default: the
              current stream); it is ordered after the current stream where it reads tensors
              made there (``init``, a default ``out``).
    tuning    launch shape, the ltl_tuning_t fields as keywords: steps_per_launch, tile_rows,
              tile_cols, waves, use_graph, persistent, lds_pad (0 = library default for the first four;
              without `tuning` the shape comes from the tuning table, or LTL_TILE).
    boundary  "dead" (ghost halo of dead cells) or "periodic" (torus; W must be a multiple of 16).
    The results never depend on `tuning`; unsupported or infeasible combinations raise LtlError.
    """

    def __init__(self, init, rule, method="cat_i8", stream=None, tuning: Optional[dict] = None,
                 boundary="dead"):
        import torch

        if isinstance(method, str):
            method = METHODS[method]
        if init.device.type != "cuda" or init.dtype != torch.uint8 or init.dim() != 2:
            raise ValueError("init must be a 2-D uint8 CUDA tensor")
        init = init.contiguous()
        self.H, self.W = int(init.shape[0]), int(init.shape[1])
        self.stream = _torch_stream(stream, init.device)
        self.rule = rule
        nbytes = ltl_buffer_bytes(self.H, self.W, make_rule(rule).R, method)
        # 256-byte aligned: torch's caching allocator hands out 512-byte aligned blocks
        self.bufs = [torch.empty(nbytes, dtype=torch.uint8, device=init.device) for _ in range(2)]
        _join_current(self.stream, init.device, [init] + self.bufs)
        self.handle = ltl_create(self.H, self.W, rule, method, self.bufs[0].data_ptr(), self.bufs[1].data_ptr(),
                                 nbytes, init.data_ptr(), init.stride(0), self.stream)
        self.device = init.device
        try:
            if boundary != "dead":
                ltl_set_boundary(self.handle, BOUNDARIES[boundary] if isinstance(boundary, str) else int(boundary))
            if tuning:
                ltl_set_tuning(self.handle, **tuning)
        except Exception:
            self.close()   # a refused boundary or tuning: release the handle before raising
            raise

    def step(self, n: int = 1) -> "Simulation":
        ltl_step(self.handle, n)
        return self

    def read(self, out=None):
        import torch

        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.uint8, device=self.device)
        _check_out(out, self.H, self.W, self.device)
        _join_current(self.stream, self.device, [out])
        ltl_read(self.handle, out.data_ptr(), out.stride(0))
        _current_after(self.stream, self.device)
        return out

    def current_padded(self):
        """The library-layout buffer holding the current state (H rows x pitch); torch's current
        stream is ordered after the work queued on the simulation's stream."""
        ptr, pitch, _ = ltl_current(self.handle)
        idx = 0 if ptr == self.bufs[0].data_ptr() else 1
        _current_after(self.stream, self.device)
        return self.bufs[idx][: self.H * pitch].view(self.H, pitch)

    @property
    def steps_done(self) -> int:
        return ltl_current(self.handle)[2]

    def tuning(self) -> dict:
        return ltl_get_tuning(self.handle).as_dict()

    def set_tuning(self, **kw) -> None:
        ltl_set_tuning(self.handle, **kw)

    def autotune(self, probe_steps: int = 8) -> dict:
        """Pick the fastest launch shape by timing on the device (the state does not advance).
        The probe's save copy is a torch tensor made here."""
        import torch

        scratch = torch.empty(self.bufs[0].numel(), dtype=torch.uint8, device=self.device)
        _join_current(self.stream, self.device, [scratch])
        return ltl_autotune(self.handle, probe_steps, scratch.data_ptr(), scratch.numel()).as_dict()

    def close(self) -> None:
        if self.handle:
            import torch

            torch.cuda.synchronize(self.device)
            ltl_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many automata advanced together; the two arenas are torch uint8 tensors on the GPU.
    ``inits``: 2-D uint8 CUDA tensors (one per instance), ``rules``: one rule per instance."""

    def __init__(self, inits, rules, method="cat_i8", stream=None, tuning: Optional[dict] = None):
        import torch

        if isinstance(method, str):
            method = METHODS[method]
        if len(inits) != len(rules) or not inits:
            raise ValueError("need one rule per initial grid, at least one instance")
        for g in inits:
            if g.device.type != "cuda" or g.dtype != torch.uint8 or g.dim() != 2 or g.stride(1) != 1:
                raise ValueError("every initial grid must be a row-major 2-D uint8 CUDA tensor")
        self.device = inits[0].device
        self.H = [int(g.shape[0]) for g in inits]
        self.W = [int(g.shape[1]) for g in inits]
        self.stream = _torch_stream(stream, self.device)
        self.nbytes = ltl_batch_buffer_bytes(self.H, self.W)
        self.arenas = [torch.empty(self.nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        _join_current(self.stream, self.device, list(inits) + self.arenas)
        self.handle = ltl_batch_create(self.H, self.W, rules, method, self.arenas[0].data_ptr(),
                                       self.arenas[1].data_ptr(), self.nbytes, [g.data_ptr() for g in inits],
                                       [g.stride(0) for g in inits], self.stream)
        if tuning:
            try:
                ltl_batch_set_tuning(self.handle, **tuning)
            except Exception:
                self.close()   # a refused tuning: release the handle before raising
                raise

    def __len__(self) -> int:
        return len(self.H)

    def step(self, n: int = 1) -> "Batch":
        ltl_batch_step(self.handle, n)
        return self

    def read(self, index: int, out=None):
        import torch

        if out is None:
            out = torch.empty((self.H[index], self.W[index]), dtype=torch.uint8, device=self.device)
        _check_out(out, self.H[index], self.W[index], self.device)
        _join_current(self.stream, self.device, [out])
        ltl_batch_read(self.handle, index, out.data_ptr(), out.stride(0))
        _current_after(self.stream, self.device)
        return out

    def current_padded(self, index: int):
        """Instance `index`'s current state in the library layout (H rows x pitch), a view."""
        ptr, pitch, _ = ltl_batch_current(self.handle, index)
        _current_after(self.stream, self.device)
        for a in self.arenas:
            off = ptr - a.data_ptr()
            if 0 <= off < self.nbytes:
                return a[off: off + self.H[index] * pitch].view(self.H[index], pitch)
        raise RuntimeError("instance buffer outside both arenas")

    @property
    def steps_done(self) -> int:
        return ltl_batch_current(self.handle, 0)[2]

    def tuning(self) -> dict:
        return ltl_batch_get_tuning(self.handle).as_dict()

    def set_tuning(self, **kw) -> None:
        ltl_batch_set_tuning(self.handle, **kw)

    def autotune(self, probe_steps: int = 4) -> dict:
        """Pick the fastest launch shape by timing on the device (the state does not advance)."""
        import torch

        scratch = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        _join_current(self.stream, self.device, [scratch])
        return ltl_batch_autotune(self.handle, probe_steps, scratch.data_ptr(), scratch.numel()).as_dict()

    def close(self) -> None:
        if self.handle:
            import torch

            torch.cuda.synchronize(self.device)
            ltl_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
