"""Host-side checks of the tuned-plan table (no GPU): the JSON reader, the lookup by
workload key and particle count, and the fall-back to the fixed rules for a tuned
shape the kernel cannot run."""
import ctypes
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNING = os.path.join(ROOT, "paper_1406_4254_amd", "etics_tuning.json")

FP64, MIXED, COMP32 = 0, 1, 2


@pytest.fixture()
def E():
    from paper_1406_4254_amd import etics
    etics.lib()
    etics.etics_tuning_clear()
    yield etics
    # leave the process with the table the library loads by itself
    if os.path.exists(TUNING):
        etics.etics_tuning_load(TUNING)
    else:
        etics.etics_tuning_clear()


def test_fixed_rules_without_a_table(E):
    for prec in (FP64, MIXED, COMP32):
        info = E.etics_plan_info(1_000_000, 10, 10, prec)
        assert not info["tuned"]
        assert info["phase2"] == 1  # outer products on the VALU by default
        assert info["tp"] >= 1 and info["grid"] >= 1


def test_set_plan_is_used_and_reported(E):
    shape = {"nw": 4, "tp": 60, "streams": 5, "grid_mult": 1, "unit": 0, "split": 0, "phase2": 1}
    E.etics_tuning_set(10, 10, MIXED, 1_000_000, shape)
    info = E.etics_plan_info(1_000_000, 10, 10, MIXED)
    assert info["tuned"]
    for k in ("nw", "tp", "streams", "grid_mult", "phase2"):
        assert info[k] == shape[k], k
    # another precision or cutoff is another key
    assert not E.etics_plan_info(1_000_000, 10, 10, FP64)["tuned"]
    assert not E.etics_plan_info(1_000_000, 10, 9, MIXED)["tuned"]
    assert not E.etics_plan_info(1_000_000, 10, 10, MIXED, batched=True)["tuned"]


def test_lookup_within_a_factor_of_8_in_n(E):
    E.etics_tuning_set(10, 6, MIXED, 100_000, {"tp": 48, "streams": 4, "phase2": 1})
    assert E.etics_plan_info(100_000 * 8, 10, 6, MIXED)["tuned"]
    assert E.etics_plan_info(100_000 // 8, 10, 6, MIXED)["tuned"]
    assert not E.etics_plan_info(100_000 * 9, 10, 6, MIXED)["tuned"]
    assert not E.etics_plan_info(100_000 // 9, 10, 6, MIXED)["tuned"]
    # the nearest entry in log2(n) wins
    E.etics_tuning_set(10, 6, MIXED, 1_000_000, {"tp": 32, "streams": 4, "phase2": 1})
    assert E.etics_plan_info(150_000, 10, 6, MIXED)["tp"] == 48
    assert E.etics_plan_info(700_000, 10, 6, MIXED)["tp"] == 32


@pytest.mark.parametrize("shape", [
    {"nw": 3},                                   # not 1, 2 or 4 wavefronts per group
    {"nw": 1, "tp": 256},                        # 1 wavefront per group only for lmax <= 6
    {"tp": 65},                                  # more than 64 particles per group of 64 lanes
    {"streams": 300},                            # more stream copies than lanes
    {"grid_mult": 3},
    {"unit": 100},                               # below the smallest work unit
    {"unit": 4096, "split": 128},                # fewer than 64 particles per force workgroup
])
def test_invalid_tuned_shape_falls_back(E, shape):
    fixed = E.etics_plan_info(1_000_000, 10, 10, MIXED)
    E.etics_tuning_set(10, 10, MIXED, 1_000_000, shape)
    info = E.etics_plan_info(1_000_000, 10, 10, MIXED)
    assert not info["tuned"]
    assert info == fixed


def test_matrix_phase2_is_fp32_only(E):
    E.etics_tuning_set(10, 10, FP64, 1_000_000, {"phase2": 2})
    assert not E.etics_plan_info(1_000_000, 10, 10, FP64)["tuned"]
    for prec in (MIXED, COMP32):
        E.etics_tuning_set(10, 10, prec, 1_000_000, {"phase2": 2})
        info = E.etics_plan_info(1_000_000, 10, 10, prec)
        assert info["tuned"] and info["phase2"] == 2


def test_set_rejects_bad_arguments(E):
    L = E.lib()
    vals = (ctypes.c_int * 7)()
    assert L.etics_tuning_set(0, 10, 10, MIXED, 0, 1000, vals, 6) < 0  # 7 parameters
    assert L.etics_tuning_set(2, 10, 10, MIXED, 0, 1000, vals, 7) < 0  # batched is 0 or 1
    assert L.etics_tuning_set(0, 10, 10, MIXED, 0, 0, vals, 7) < 0     # n >= 1
    assert L.etics_tuning_set(0, 10, 10, MIXED, 0, 1000, None, 7) < 0


def test_load_json(E, tmp_path):
    doc = {"device": "x", "plans": [
        {"batched": 0, "nmax": 10, "lmax": 10, "prec": MIXED, "basis": 0, "n": 1000000,
         "nw": 4, "tp": 56, "streams": 7, "grid_mult": 2, "unit": 4096, "split": 4, "phase2": 1,
         "ms": 0.1, "note": "strings and other keys are ignored"},
        {"batched": 1, "nmax": 8, "lmax": 6, "prec": FP64, "n": 5500000,
         "nw": 4, "tp": 64, "streams": 16, "grid_mult": 2, "unit": 2048, "split": 2, "phase2": 1},
        {"nmax": 10, "lmax": 6, "n": 1000, "tp": 1.5},  # not an integer: skipped
    ]}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(doc))
    assert E.etics_tuning_load(str(f)) == 2
    info = E.etics_plan_info(1_000_000, 10, 10, MIXED)
    assert info["tuned"] and info["tp"] == 56 and info["streams"] == 7
    b = E.etics_plan_info(5_500_000, 8, 6, FP64, batched=True)
    assert b["tuned"] and b["unit"] == 2048 and b["split"] == 2
    # a load replaces the table
    f2 = tmp_path / "u.json"
    f2.write_text(json.dumps({"plans": []}))
    assert E.etics_tuning_load(str(f2)) == 0
    assert not E.etics_plan_info(1_000_000, 10, 10, MIXED)["tuned"]


def test_load_errors(E, tmp_path):
    with pytest.raises(RuntimeError):
        E.etics_tuning_load(str(tmp_path / "missing.json"))
    bad = tmp_path / "bad.json"
    bad.write_text('{"plans": [{"nmax": 10, "lmax": ')
    with pytest.raises(RuntimeError):
        E.etics_tuning_load(str(bad))


def test_committed_table_is_valid(E):
    """Every plan of the table shipped next to the library is in force for its own key."""
    if not os.path.exists(TUNING):
        pytest.skip("no tuned table committed")
    with open(TUNING) as fh:
        plans = json.load(fh)["plans"]
    assert E.etics_tuning_load(TUNING) == len(plans) > 0
    for p in plans:
        info = E.etics_plan_info(p["n"], p["nmax"], p["lmax"], p["prec"], batched=bool(p.get("batched", 0)),
                                 basis=p.get("basis", 0))
        assert info["tuned"], p
        for k in E.PLAN_FIELDS:
            if p.get(k, 0):
                assert info[k] == p[k], (k, p)
