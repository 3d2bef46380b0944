"""CPU checks of the benchmark script's contract: one GPU only, the per-pair byte table it prices the
roofline with, and the rule that counter-derived traffic is reported only for the kernel source it
was measured on."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bytes_per_pair_follow_the_stored_state():
    """Bytes per pair of the dominant pass, re-derived from the element sizes: the constant step and
    the re-forming trial passes read H (none in FP64) and two stored iterates and write one; the
    FP64 storing trial reads two iterates and writes both candidates."""
    b = _bench()
    hi = {"fp64": 0, "mixed_fp32": 4, "mixed_bf16": 2}
    it = {"fp64": 8, "mixed_fp32": 4, "mixed_bf16": 4}
    for p in hi:
        assert b.PASS_BYTES[("constant", p)] == hi[p] + 3 * it[p]
    for p in ("mixed_fp32", "mixed_bf16"):
        assert b.PASS_BYTES[("adaptive", p)] == hi[p] + 3 * it[p]
    assert b.PASS_BYTES[("adaptive", "fp64_reform")] == 3 * it["fp64"]
    assert b.PASS_BYTES[("adaptive", "fp64")] == 4 * it["fp64"]
    assert b.pass_kernel("adaptive", "mixed_fp32") == "pass_kernel<float,REP_SPLIT_F32,PASS_ADV,MB=3,KT=2>"
    assert b.pass_kernel("adaptive", "fp64") == "pass_kernel<double,REP_F64,PASS_TRIAL,MB=3,KT=2>"
    assert b.pass_kernel("constant", "fp64") == "pass_kernel<double,REP_F64,PASS_STEP,MB=3,KT=2>"


def test_traffic_only_for_the_measured_kernel_source(tmp_path, monkeypatch):
    b = _bench()
    label = b.pass_kernel("adaptive", "mixed_fp32")
    entry = {"bytes_per_launch": 1.0e9}
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"kernel_source_sha256_16": b.kernel_hash(), "kernels": {label: entry}}))
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"kernel_source_sha256_16": "0" * 16, "kernels": {label: entry}}))
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(good))
    assert b.traffic_for(label) == entry
    assert b.traffic_for("pass_kernel<other>") is None
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(stale))
    assert b.traffic_for(label) is None
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert b.traffic_for(label) is None


@pytest.mark.parametrize("name", ["pass_traffic_quad_N8000_n40.json"])
def test_committed_traffic_file_is_well_formed(name):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        t = json.load(f)
    assert len(t["kernel_source_sha256_16"]) == 16 and "rocprofv3" in t["how"]
    for k in t["kernels"].values():
        assert k["bytes_per_launch"] == pytest.approx(k["fetch_bytes"] + k["write_bytes"])
        assert k["bytes_per_launch"] >= k["algorithmic_bytes_per_launch"]


def test_line_stays_short_and_keeps_the_contract():
    """The driver keeps a bounded tail of stdout: the JSON line is cut to LINE_LIMIT characters by
    dropping optional sections (named in the line), never the contract's fields."""
    b = _bench()
    core = {"metric": "m", "value": 1.0, "unit": "u", "n_gpus": 1, "steps": 2, "warmup": 1, "ms_per_step": 1.0,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
            "data": "synthetic", "config": {"workload": "w"},
            "roofline": {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.5,
                         "traffic": None},
            "cpu_baseline": {"value": 1.0, "unit": "u", "cores": 16, "kind": "oracle", "sample": "s"}}
    short = b.render_line(core)
    assert json.loads(short) == core
    big = dict(core)
    for key in b.OPTIONAL_ORDER:
        big[key] = {"pad": "x" * 1500}
    line = b.render_line(big)
    assert len(line) <= b.LINE_LIMIT
    got = json.loads(line)
    for key in core:
        assert got[key] == core[key]
    assert got["dropped_for_length"] and all(k not in got for k in got["dropped_for_length"])
    # sections are dropped in the stated order, and only as many as needed
    kept = [k for k in b.OPTIONAL_ORDER if k in got]
    assert got["dropped_for_length"] == [k for k in b.OPTIONAL_ORDER if k not in kept]
    assert kept == b.OPTIONAL_ORDER[len(got["dropped_for_length"]):]
