"""Host logic of bench.py (no GPU): launch-shape parsing, the counter records it reads only
while they match the kernel source and launch shape, the counter-based MFMA utilisation
arithmetic, and the one-GPU refusal."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

DEFAULT = dict(steps_per_launch=4, tile_rows=160, tile_cols=224, waves=8, persistent=0, lds_pad=0)


def test_parse_tuning():
    assert bench.parse_tuning("4,160,224,8") == dict(steps_per_launch=4, tile_rows=160, tile_cols=224, waves=8)
    assert bench.parse_tuning("1,64,128,4,1")["persistent"] == 1
    assert bench.parse_tuning("1,64,128,4,0,32")["lds_pad"] == 32


def write_record(tmp_path, **fields):
    rec = dict(kernel_sha256=bench.kernel_hash(), tuning=[DEFAULT[k] for k in bench.SHAPE_KEYS], **fields)
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    return str(path)


def test_records_are_used_only_for_the_kernel_and_shape_they_were_taken_on(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", write_record(tmp_path, hbm_bytes_per_launch=123.0))
    assert bench.recorded_traffic(DEFAULT) == 123.0
    assert bench.recorded_traffic(dict(DEFAULT, tile_rows=128)) is None
    assert bench.recorded_traffic(dict(DEFAULT, persistent=1)) is None
    assert bench.recorded_traffic(dict(DEFAULT, lds_pad=16)) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "another kernel")
    assert bench.recorded_traffic(DEFAULT) is None
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "missing.json"))
    assert bench.recorded_traffic(DEFAULT) is None


def test_mfma_issued_arithmetic(tmp_path, monkeypatch):
    cells = 4096 * 4096
    ops = 375.0 * cells * 4          # 375 int8 ops issued per cell-update, 4 steps per launch
    monkeypatch.setattr(bench, "MFMA_RECORD", write_record(tmp_path, mfma_ops_per_launch=ops))
    m = bench.mfma_issued(DEFAULT, 25e-6, cells, 5)
    assert m["issued_ops_per_cell_update"] == pytest.approx(375.0)
    assert m["useful_ops_per_cell_update"] == 44
    assert m["useful_frac"] == pytest.approx(44 / 375.0)
    assert m["frac_of_peak"] == pytest.approx(ops / 25e-6 / 5e15)
    assert bench.mfma_issued(dict(DEFAULT, steps_per_launch=2), 25e-6, cells, 5) is None


def test_committed_records_are_well_formed():
    for name, key in (("cat_step_i8_bosco4096_traffic.json", "hbm_bytes_per_launch"),
                      ("cat_step_i8_bosco4096_sq.json", "mfma_ops_per_launch")):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            rec = json.load(f)
        assert len(rec["kernel_sha256"]) == 64
        assert 5 <= len(rec["tuning"]) <= len(bench.SHAPE_KEYS)
        assert rec[key] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_records_without_the_pad_field_read_as_pad_zero(tmp_path, monkeypatch):
    """Records taken before the LDS row padding knob existed hold five shape fields."""
    rec = dict(kernel_sha256=bench.kernel_hash(), tuning=[4, 160, 224, 8, 0], hbm_bytes_per_launch=7.0)
    path = tmp_path / "old.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(path))
    assert bench.recorded_traffic(DEFAULT) == 7.0
    assert bench.recorded_traffic(dict(DEFAULT, lds_pad=32)) is None


def test_median_timing_restarts_every_repetition():
    """time_reps resets the state before every timed run and times each run on its own."""
    calls = []

    class Ev:
        def __init__(self, enable_timing=True):
            self.t = 0.0

        def record(self, stream):
            calls.append(("record", stream))
            self.t = len(calls)

        def elapsed_time(self, other):
            return (other.t - self.t) * 1000.0

    class FakeTorch:
        class cuda:
            Event = Ev

            @staticmethod
            def synchronize():
                calls.append(("sync", None))

    times = bench.time_reps("s", lambda: calls.append(("run", None)), lambda: calls.append(("reset", None)), 3,
                            FakeTorch)
    assert len(times) == 3
    kinds = [c[0] for c in calls]
    assert kinds == ["reset", "sync", "record", "run", "record", "sync"] * 3
