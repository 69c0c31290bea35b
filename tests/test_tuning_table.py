"""Tuning table (no GPU): keys, lookup order, the user cache and the shipped table.

The library reads two JSON files at every lookup: the user cache (LTL_TUNE_CACHE) first, then
the table shipped beside it (LTL_TUNE_TABLE overrides its path). These tests point both at
files of their own."""
import json
import os

import pytest

from paper_2406_17284_amd import inputs, ltl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIPPED = os.path.join(ROOT, "paper_2406_17284_amd", "tuning.json")

BOSCO = inputs.BOSCO_M1


def entry(method="cat_i8", elem="i8", epi="byte", r=5, bucket=12, boundary="dead", batched=0,
          tuning=(4, 160, 224, 8, 1, 0, 0), ms=0.01):
    return {"method": method, "elem": elem, "epi": epi, "r": r, "bucket": bucket, "boundary": boundary,
            "batched": batched, "tuning": list(tuning), "ms_per_step": ms}


def write(path, entries):
    path.write_text(json.dumps({"version": 1, "entries": entries}))


@pytest.fixture
def files(tmp_path, monkeypatch):
    user = tmp_path / "user.json"
    table = tmp_path / "table.json"
    monkeypatch.setenv("LTL_TUNE_CACHE", str(user))
    monkeypatch.setenv("LTL_TUNE_TABLE", str(table))
    return user, table


def shape(t):
    return (t.steps_per_launch, t.tile_rows, t.tile_cols, t.waves, t.use_graph, t.persistent, t.lds_pad)


def test_exact_key(files):
    user, table = files
    write(table, [entry(), entry(r=6, epi="win", tuning=(3, 128, 192, 8, 1, 0, 16))])
    t, exact = ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8)
    assert exact and shape(t) == (4, 160, 224, 8, 1, 0, 0)
    # the sweep rule of radius 6 is a windowed-epilogue rule: the "win" entry of r = 6
    t, exact = ltl.ltl_tuning_lookup(4096, 4096, inputs.sweep_rule(6), ltl.LTL_CAT_I8)
    assert exact and shape(t) == (3, 128, 192, 8, 1, 0, 16)


def test_size_bucket_is_log2_of_the_side(files):
    user, table = files
    write(table, [entry(bucket=b, tuning=(b, 16 * b, 32, 1, 1, 0, 0)) for b in (8, 12, 14, 15)])
    for side, b in ((256, 8), (4096, 12), (16384, 14), (32768, 15), (5000, 12), (6000, 13)):
        t, exact = ltl.ltl_tuning_lookup(side, side, BOSCO, ltl.LTL_CAT_I8)
        if side == 6000:   # log2(6000) = 12.55 -> bucket 13, no entry: nearest are 12 and 14, 12 first in the file
            assert not exact and t.steps_per_launch in (12, 14)
        else:
            assert exact and t.steps_per_launch == b, side
    # rectangular grids use the cell count: 2048 x 32768 has the cells of 8192^2 (bucket 13)
    t, exact = ltl.ltl_tuning_lookup(2048, 32768, BOSCO, ltl.LTL_CAT_I8)
    assert not exact


def test_nearest_radius_then_nearest_bucket(files):
    user, table = files
    write(table, [entry(r=4, bucket=14, tuning=(1, 64, 64, 1, 1, 0, 0)),
                  entry(r=5, bucket=8, tuning=(2, 64, 64, 1, 1, 0, 0)),
                  entry(r=5, bucket=15, tuning=(3, 64, 64, 1, 1, 0, 0))])
    # same radius beats nearer bucket of another radius; among r = 5, bucket 15 is nearer to 12 than 8
    t, exact = ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8)
    assert not exact and t.steps_per_launch == 3


def test_user_cache_first_and_class_must_match(files):
    user, table = files
    write(table, [entry(tuning=(1, 64, 64, 1, 1, 0, 0))])
    write(user, [entry(tuning=(2, 64, 64, 1, 1, 0, 0))])
    t, _ = ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8)
    assert t.steps_per_launch == 2
    # entries of another class are never used
    write(user, [])
    write(table, [entry(method="cat_f16", elem="f16"), entry(boundary="periodic"), entry(batched=1, epi="mixed", r=0),
                  entry(epi="half"), entry(elem="i8x")])
    assert ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8) is None
    t, exact = ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8, ltl.LTL_BOUNDARY_PERIODIC)
    assert exact


@pytest.mark.parametrize("rule,method,elem,epi", [
    (inputs.BOSCO_M1, ltl.LTL_CAT_I8, "i8", "byte"),           # counts <= 121 fit bytes
    (inputs.sweep_rule(6), ltl.LTL_CAT_I8, "i8", "win"),       # ranges inside a 126-wide window
    (inputs.sweep_rule(13), ltl.LTL_CAT_I8, "i8", "win"),      # ranges inside a 254-wide window
    (inputs.Rule(13, 0, 1, 100, 500, 150, 300), ltl.LTL_CAT_I8, "i8", "half"),   # wider than 254
    (inputs.DECAY_C8, ltl.LTL_CAT_I8, "i8", "decay"),
    (inputs.sweep_rule(6), ltl.LTL_CAT_F16, "f16", "half"),    # windowed bytes are int8 only
    (inputs.sweep_rule(5), ltl.LTL_CAT_F8, "f8", "byte"),
    (inputs.Rule(20, 0, 1, 400, 700, 420, 600), ltl.LTL_CAT_I8, "i8w", "half"),
    (inputs.Rule(3, 0, 1, 3, 6, 3, 4, "N"), ltl.LTL_CAT_I8, "i8x", "byte"),
    (inputs.BOSCO_M1, ltl.LTL_DIRECT, "direct", "byte"),
])
def test_key_classes(files, rule, method, elem, epi):
    user, table = files
    write(table, [entry(method={0: "cat_i8", 1: "cat_f16", 2: "cat_f8", 3: "direct"}[method], elem=elem, epi=epi,
                        r=rule.R)])
    got = ltl.ltl_tuning_lookup(4096, 4096, rule, method)
    assert got is not None and got[1], (elem, epi)


def test_batched_key(files):
    user, table = files
    insts = inputs.batch_instances(count=8)
    cells = sum(x.H * x.W for x in insts)
    rmax = max(x.rule.R for x in insts)
    write(table, [entry(batched=1, epi="mixed", r=0, bucket=14, tuning=(3, 160, 160, 8, 1, 0, 0))])
    rule = inputs.Rule(rmax, 0, 1, 0, 0, 0, 0)
    t, exact = ltl.ltl_tuning_lookup(cells, 1, rule, ltl.LTL_CAT_I8, batched=1)
    assert shape(t)[:4] == (3, 160, 160, 8)


def test_store_inserts_and_replaces(files):
    user, table = files
    assert not user.exists()
    ltl.ltl_tuning_store(4096, 4096, BOSCO, ltl.LTL_CAT_I8, 0, 0, dict(steps_per_launch=4, tile_rows=160,
                         tile_cols=224, waves=8, use_graph=1, persistent=0, lds_pad=32), 0.0066)
    data = json.loads(user.read_text())
    assert len(data["entries"]) == 1
    e = data["entries"][0]
    assert (e["method"], e["elem"], e["epi"], e["r"], e["bucket"], e["boundary"], e["batched"]) == \
        ("cat_i8", "i8", "byte", 5, 12, "dead", 0)
    assert e["tuning"] == [4, 160, 224, 8, 1, 0, 32]
    ltl.ltl_tuning_store(4096, 4096, BOSCO, ltl.LTL_CAT_I8, 0, 0, dict(steps_per_launch=3, tile_rows=128,
                         tile_cols=192, waves=8, use_graph=1), 0.007)
    ltl.ltl_tuning_store(16384, 16384, BOSCO, ltl.LTL_CAT_I8, 0, 0, dict(steps_per_launch=5, tile_rows=128,
                         tile_cols=192, waves=8, use_graph=1), 0.1)
    data = json.loads(user.read_text())
    assert len(data["entries"]) == 2   # same key replaced, new bucket added
    t, exact = ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8)
    assert exact and t.steps_per_launch == 3


def test_store_refused_when_cache_is_off(monkeypatch):
    monkeypatch.setenv("LTL_TUNE_CACHE", "off")
    with pytest.raises(ltl.LtlError) as e:
        ltl.ltl_tuning_store(64, 64, BOSCO, ltl.LTL_CAT_I8, 0, 0, dict(steps_per_launch=1), 1.0)
    assert e.value.code == ltl.LTL_ERR_ARG


def test_malformed_files_are_ignored(files):
    user, table = files
    user.write_text("{not json")
    write(table, [{"method": "cat_i8"}, entry(tuning=(1, 2)), entry(tuning=(2, 64, 64, 1, 1, 0, 0))])
    t, exact = ltl.ltl_tuning_lookup(4096, 4096, BOSCO, ltl.LTL_CAT_I8)
    assert exact and t.steps_per_launch == 2


def test_lookup_rejects_bad_arguments(files):
    with pytest.raises(ltl.LtlError):
        ltl.ltl_tuning_lookup(0, 4, BOSCO, ltl.LTL_CAT_I8)
    with pytest.raises(ltl.LtlError) as e:
        ltl.ltl_tuning_lookup(4, 4, inputs.Rule(8, 0, 1, 3, 4, 3, 3), ltl.LTL_CAT_F8)
    assert e.value.code == ltl.LTL_ERR_INEXACT


def test_shipped_table_covers_the_benchmark_workloads(monkeypatch):
    """The table beside the library parses, every entry is well formed, and the benchmark's
    workloads find exact entries (so a fresh Simulation runs them at the tuned shape)."""
    monkeypatch.setenv("LTL_TUNE_CACHE", "off")
    monkeypatch.delenv("LTL_TUNE_TABLE", raising=False)
    data = json.load(open(SHIPPED))
    keys = set()
    for e in data["entries"]:
        k = (e["method"], e["elem"], e["epi"], e["r"], e["bucket"], e["boundary"], e["batched"])
        assert k not in keys, k
        keys.add(k)
        assert len(e["tuning"]) == 7
        T, th, tw, wv, graph, pers, pad = e["tuning"]
        assert 1 <= T <= 64 and th % 16 == 0 and tw % 32 == 0 and 1 <= wv <= 16 and pad % 16 == 0
    w = inputs.WORKLOADS["bosco4096"]
    assert ltl.ltl_tuning_lookup(w.H, w.W, w.rule, ltl.LTL_CAT_I8)[1]
    w = inputs.WORKLOADS["decay32768"]
    assert ltl.ltl_tuning_lookup(w.H, w.W, w.rule, ltl.LTL_CAT_I8)[1]
    w = inputs.WORKLOADS["life256"]
    assert ltl.ltl_tuning_lookup(w.H, w.W, w.rule, ltl.LTL_CAT_I8)[1]
    for r in range(1, 17):
        w = inputs.sweep_workload(r)
        assert ltl.ltl_tuning_lookup(w.H, w.W, w.rule, ltl.LTL_CAT_I8)[1], r
        assert ltl.ltl_tuning_lookup(w.H, w.W, w.rule, ltl.LTL_CAT_F16)[1], r
        if r <= 7:
            assert ltl.ltl_tuning_lookup(w.H, w.W, w.rule, ltl.LTL_CAT_F8)[1], r
    insts = inputs.batch_instances()
    cells = sum(x.H * x.W for x in insts)
    rule = inputs.Rule(max(x.rule.R for x in insts), 0, 1, 0, 0, 0, 0)
    assert ltl.ltl_tuning_lookup(cells, 1, rule, ltl.LTL_CAT_I8, batched=1)[1]
