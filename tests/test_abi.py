"""C-ABI contract checks that need no GPU: the library loads, exports every function
declared in include/ltl.h, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2406_17284_amd import ltl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ltl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ltl_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = ltl.load()
    names = declared_functions()
    assert len(names) >= 16
    assert sorted(ltl.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_pitch_and_buffer_bytes():
    assert ltl.ltl_pitch(1) == 64
    assert ltl.ltl_pitch(64) == 64
    assert ltl.ltl_pitch(65) == 128
    # the halo is not stored: the size depends on neither the radius nor the method
    for R in (1, 16, 32):
        for m in (ltl.LTL_CAT_I8, ltl.LTL_CAT_F16, ltl.LTL_CAT_F8, ltl.LTL_DIRECT):
            assert ltl.ltl_buffer_bytes(3, 100, R, m) == 3 * 128
    for bad, code in [((0, 5, 1, 0), ltl.LTL_ERR_ARG), ((5, 0, 1, 0), ltl.LTL_ERR_ARG), ((-1, 3, 1, 0), ltl.LTL_ERR_ARG),
                      ((3, 3, 0, 0), ltl.LTL_ERR_RULE), ((3, 3, 33, 0), ltl.LTL_ERR_RULE), ((3, 3, 1, 4), ltl.LTL_ERR_ARG),
                      ((3, 3, 1, -1), ltl.LTL_ERR_ARG)]:
        with pytest.raises(ltl.LtlError) as e:
            ltl.ltl_buffer_bytes(*bad)
        assert e.value.code == code, bad
        assert ltl.load().ltl_last_error_code() == code
        assert ltl.last_error()


def _create(H=8, W=8, rule=(1, 0, 1, 3, 4, 3, 3), method=ltl.LTL_CAT_I8, a=256, b=512, nbytes=1 << 20, init=1024,
            pitch=8):
    return ltl.ltl_create(H, W, rule, method, a, b, nbytes, init, pitch)


@pytest.mark.parametrize("kw,code", [
    (dict(H=0), ltl.LTL_ERR_ARG),
    (dict(a=0), ltl.LTL_ERR_ARG),
    (dict(init=0), ltl.LTL_ERR_ARG),
    (dict(a=256, b=256), ltl.LTL_ERR_ARG),
    (dict(pitch=4), ltl.LTL_ERR_ARG),
    (dict(a=100), ltl.LTL_ERR_ARG),
    (dict(rule=(0, 0, 1, 3, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(33, 0, 1, 3, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(17, 0, 1, 3, 4, 3, 3), method=ltl.LTL_CAT_F16), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rule=(1, 1, 1, 3, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(1, 256, 1, 3, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(1, 0, 2, 3, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(1, 0, 1, -1, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(1, 0, 1, 3, 10, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(rule=(2, 0, 1, 3, 4, 3, 3, "X")), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rule=(2, 0, 1, 3, 4, 3, 3, "N"), method=ltl.LTL_CAT_F16), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rule=(17, 0, 1, 3, 4, 3, 3, "N")), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rule=(8, 0, 1, 3, 4, 3, 3), method=ltl.LTL_CAT_F8), ltl.LTL_ERR_INEXACT),
    (dict(method=7), ltl.LTL_ERR_ARG),
    (dict(nbytes=63), ltl.LTL_ERR_SIZE),
    (dict(H=32768, W=65536, nbytes=1 << 31, pitch=65536), ltl.LTL_ERR_SIZE),   # 2^31 bytes: too large
])
def test_create_rejects_bad_arguments(kw, code):
    with pytest.raises(ltl.LtlError) as e:
        _create(**kw)
    assert e.value.code == code
    assert ltl.last_error()


def test_null_handles():
    lib = ltl.load()
    assert lib.ltl_step(None, 1) == ltl.LTL_ERR_ARG
    assert lib.ltl_read(None, None, 0) == ltl.LTL_ERR_ARG
    assert lib.ltl_destroy(None) == ltl.LTL_OK
    assert lib.ltl_batch_destroy(None) == ltl.LTL_OK
    assert lib.ltl_set_boundary(None, ltl.LTL_BOUNDARY_PERIODIC) == ltl.LTL_ERR_ARG
    t = ltl.ltl_tuning_t()
    assert lib.ltl_get_tuning(None, ctypes.byref(t)) == ltl.LTL_ERR_ARG
    assert lib.ltl_autotune(None, 1, None, 0, None) == ltl.LTL_ERR_ARG


def test_malformed_tile_override_is_refused_before_device_work(monkeypatch):
    """LTL_TILE is parsed before ltl_create touches the device: a malformed value is LTL_ERR_ARG."""
    for bad in ("4,160", "a,b,c,d", "4,160,224,8,0,0,9", "4;160;224;8", "-1,16,32,1"):
        monkeypatch.setenv("LTL_TILE", bad)
        with pytest.raises(ltl.LtlError) as e:
            _create()
        assert e.value.code == ltl.LTL_ERR_ARG
        assert "LTL_TILE" in ltl.last_error()


def test_batch_buffer_bytes():
    # each instance: H rows at the 64-byte pitch, rounded up to 256 bytes
    assert ltl.ltl_batch_buffer_bytes([3], [100]) == 512
    assert ltl.ltl_batch_buffer_bytes([3, 1, 8], [100, 1, 64]) == 512 + 256 + 512
    for H, W in [([], []), ([0], [4]), ([4, 5], [4, -1])]:
        with pytest.raises(ltl.LtlError) as e:
            ltl.ltl_batch_buffer_bytes(H, W)
        assert e.value.code == ltl.LTL_ERR_ARG


def _batch_create(H=(8, 8), W=(8, 8), rules=((1, 0, 1, 3, 4, 3, 3), (2, 3, 0, 5, 9, 4, 7)), method=ltl.LTL_CAT_I8,
                  a=256, b=512, nbytes=1 << 20, inits=(1024, 2048), pitches=(8, 8)):
    return ltl.ltl_batch_create(list(H), list(W), list(rules), method, a, b, nbytes, list(inits), list(pitches))


@pytest.mark.parametrize("kw,code", [
    (dict(a=0), ltl.LTL_ERR_ARG),
    (dict(a=256, b=256), ltl.LTL_ERR_ARG),
    (dict(a=100), ltl.LTL_ERR_ARG),
    (dict(inits=(1024, 0)), ltl.LTL_ERR_ARG),
    (dict(pitches=(8, 7)), ltl.LTL_ERR_ARG),
    (dict(H=(8, 0)), ltl.LTL_ERR_ARG),
    (dict(rules=((1, 0, 1, 3, 4, 3, 3), (33, 0, 1, 3, 4, 3, 3))), ltl.LTL_ERR_RULE),
    (dict(rules=((1, 0, 1, 3, 4, 3, 3), (17, 0, 1, 3, 4, 3, 3))), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rules=((1, 0, 1, 3, 4, 3, 3), (1, 0, 1, 3, 4, 3, 3, "X"))), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rules=((1, 0, 1, 3, 4, 3, 3), (1, 0, 1, 3, 4, 3, 3, "N"))), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rules=((7, 0, 1, 3, 4, 3, 3), (8, 0, 1, 3, 4, 3, 3)), method=ltl.LTL_CAT_F8), ltl.LTL_ERR_INEXACT),
    (dict(method=9), ltl.LTL_ERR_ARG),
    (dict(nbytes=1023), ltl.LTL_ERR_SIZE),
    (dict(H=(8, 46341), W=(8, 46341), pitches=(8, 46341), nbytes=1 << 33), ltl.LTL_ERR_SIZE),
])
def test_batch_create_rejects_bad_arguments(kw, code):
    with pytest.raises(ltl.LtlError) as e:
        _batch_create(**kw)
    assert e.value.code == code
    assert ltl.last_error()


def test_batch_null_handles():
    lib = ltl.load()
    assert lib.ltl_batch_step(None, 1) == ltl.LTL_ERR_ARG
    assert lib.ltl_batch_read(None, 0, None, 0) == ltl.LTL_ERR_ARG
    assert lib.ltl_batch_current(None, 0, None, None, None) == ltl.LTL_ERR_ARG
    t = ltl.ltl_tuning_t()
    assert lib.ltl_batch_get_tuning(None, ctypes.byref(t)) == ltl.LTL_ERR_ARG
    assert lib.ltl_batch_set_tuning(None, ctypes.byref(t)) == ltl.LTL_ERR_ARG
    assert lib.ltl_batch_autotune(None, 1, None, 0, None) == ltl.LTL_ERR_ARG


@pytest.mark.parametrize("kw,code", [
    (dict(H=0), ltl.LTL_ERR_ARG),
    (dict(a=0), ltl.LTL_ERR_ARG),
    (dict(dst=0), ltl.LTL_ERR_ARG),
    (dict(a=256, b=256), ltl.LTL_ERR_ARG),
    (dict(dst_pitch=4), ltl.LTL_ERR_ARG),
    (dict(n=-1), ltl.LTL_ERR_ARG),
    (dict(a=100), ltl.LTL_ERR_ARG),
    (dict(boundary=2), ltl.LTL_ERR_ARG),
    (dict(boundary=1, W=8), ltl.LTL_ERR_UNSUPPORTED),
    (dict(rule=(0, 0, 1, 3, 4, 3, 3)), ltl.LTL_ERR_RULE),
    (dict(method=ltl.LTL_CAT_F8, rule=(8, 0, 1, 3, 4, 3, 3)), ltl.LTL_ERR_INEXACT),
    (dict(nbytes=10), ltl.LTL_ERR_SIZE),
])
def test_run_noalloc_refusals_without_device_work(kw, code):
    """ltl_run_noalloc checks its arguments before it touches the device (no GPU needed)."""
    args = dict(H=8, W=8, rule=(1, 0, 1, 3, 4, 3, 3), method=ltl.LTL_CAT_I8, boundary=0, a=256, b=512,
                nbytes=1 << 20, init=1024, init_pitch=8, n=3, dst=2048, dst_pitch=8)
    args.update(kw)
    with pytest.raises(ltl.LtlError) as e:
        ltl.ltl_run_noalloc(args["H"], args["W"], args["rule"], args["method"], args["boundary"], args["a"], args["b"],
                            args["nbytes"], args["init"], args["init_pitch"], args["n"], args["dst"],
                            args["dst_pitch"])
    assert e.value.code == code
