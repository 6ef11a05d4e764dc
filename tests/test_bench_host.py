"""Host logic of bench.py on the CPU: the single-GPU guard, the rocprofv3 CSV summaries, the
calibrated HBM-traffic file and its source-hash check, and the kernel-resource lookup.  Inputs are
small synthetic CSV / JSON files written here."""
import csv
import json
import os
import types

import pytest

import bench


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


COPY = "lbrr::(anonymous namespace)::k_copy(unsigned int __vector(4) const*, unsigned int __vector(4)*, unsigned long)"
STEP = "void lbrr::k_step<lbrr::D3Q27, 4, float>(float const*, float*, lbrr::StepArgs)"


def _counter_runs(tmp_path, fetch_copy, write_copy, fetch_step, write_step):
    f = tmp_path / "fetch"
    w = tmp_path / "write"
    _write_csv(str(f / "x" / "fetch_counter_collection.csv"),
               [{"Kernel_Name": COPY, "Counter_Name": "FETCH_SIZE", "Counter_Value": fetch_copy}] * 3
               + [{"Kernel_Name": STEP, "Counter_Name": "FETCH_SIZE", "Counter_Value": fetch_step}] * 2)
    _write_csv(str(w / "x" / "write_counter_collection.csv"),
               [{"Kernel_Name": COPY, "Counter_Name": "WRITE_SIZE", "Counter_Value": write_copy}] * 3
               + [{"Kernel_Name": STEP, "Counter_Name": "WRITE_SIZE", "Counter_Value": write_step}] * 2)
    return str(f), str(w)


def test_traffic_is_calibrated_by_the_copy(tmp_path):
    # the copy moves 1 GiB each way; FETCH_SIZE reads half of that, WRITE_SIZE all of it (KiB)
    gib_kib = (1 << 30) / 1024
    alg = 216 * 256**3
    f, w = _counter_runs(tmp_path, gib_kib / 2, gib_kib, alg / 2 / 2 / 1024, alg / 2 / 1024)
    out = bench.write_traffic(f, w, str(tmp_path / "traffic.json"))
    assert out["copy_calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert out["copy_calibration"]["write_factor"] == pytest.approx(1.0)
    assert out["fp32"]["bytes_per_launch"] == pytest.approx(alg, rel=1e-9)
    assert out["fp32"]["ratio"] == pytest.approx(1.0)
    assert json.load(open(tmp_path / "traffic.json"))["source_hash"] == bench.kernel_source_hash()


def test_traffic_is_ignored_when_the_kernel_sources_changed(tmp_path, monkeypatch):
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"source_hash": bench.kernel_source_hash(), "fp32": {"bytes_per_launch": 123}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic("fp32") == 123
    assert bench.measured_traffic("fp16") is None
    p.write_text(json.dumps({"source_hash": "0" * 16, "fp32": {"bytes_per_launch": 123}}))
    assert bench.measured_traffic("fp32") is None


def test_profile_summary_lists_kernels_and_counters(tmp_path):
    _write_csv(str(tmp_path / "t" / "trace_kernel_stats.csv"),
               [{"Name": STEP, "Calls": "110", "AverageNs": "608410", "MinNs": "599210", "MaxNs": "675760"}])
    f, _ = _counter_runs(tmp_path, 10.0, 20.0, 30.0, 40.0)
    text = bench.summarize_prof([str(tmp_path / "t"), f])
    assert "calls    110 avg_us     608.41" in text
    step_line = [l for l in text.splitlines() if "FETCH_SIZE" in l and "k_step" in l][0]
    assert "dispatches    2" in step_line and "mean             30.0" in step_line


def test_kernel_resources_lookup(tmp_path):
    res = {STEP: {"VGPRs": 39, "Occupancy [waves/SIMD]": 8},
           "_ZN4lbrr6k_stepINS_5D3Q27ELi4EDF16_EEvPKT1_PS2_NS_8StepArgsE": {"VGPRs": 40}}
    p = tmp_path / "res.json"
    p.write_text(json.dumps(res))
    B = types.SimpleNamespace(RESOURCES=str(p))
    assert bench.kernel_resources(B, "fp32") == {"kernel": STEP, "VGPRs": 39, "Occupancy [waves/SIMD]": 8}
    assert bench.kernel_resources(B, "fp16")["VGPRs"] == 40
    assert bench.kernel_resources(B, "fp64") is None
    assert bench.kernel_resources(types.SimpleNamespace(RESOURCES=str(tmp_path / "missing.json")), "fp32") is None


@pytest.mark.parametrize("spec", ["D2Q9:4", "D3Q27", "D3Q19:x", "D3Q27:4,Q9:2"])
def test_probe_lattices_are_checked_before_any_device_work(spec, capsys):
    assert bench.main(["--probe", "--probe-lattices", spec]) == 2
    assert "bad --probe-lattices entry" in capsys.readouterr().err
