"""Host-side parts of the benchmark contract: the one-GPU refusal of
`--gpus N` and the arithmetic that turns the two counter passes (FETCH_SIZE,
WRITE_SIZE, KiB per dispatch) into HBM bytes per launch, each counter scaled
by its own reading on a 1 GiB device copy."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _counter_csv(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (name, v) in enumerate(rows):
            fh.write(f'{i},"{name}",{counter},{v}\n')


@pytest.mark.parametrize("workload", ["convdiff3d_256_exp_8rhs", "lap3d_80_invsqrt"])
def test_counter_summary_scales_each_counter_by_the_copy(tmp_path, monkeypatch, workload):
    cfg = dict(bench.BENCH[workload])
    cfg["traffic_file"] = str(tmp_path / "traffic.json")
    monkeypatch.setitem(bench.BENCH, workload, cfg)
    k = cfg["pmc_kernel"]
    # a 1 GiB copy that FETCH_SIZE sees as half its bytes and WRITE_SIZE as all
    # of them; three dispatches of the kernel and one unrelated kernel
    fetch_cal, write_cal = 524288.0, 1048576.0
    _counter_csv(tmp_path / "f", "FETCH_SIZE",
                 [("__amd_rocclr_copyBuffer", fetch_cal), (k, 1000.0), (k, 2000.0), (k, 3000.0), ("other", 9e9)])
    _counter_csv(tmp_path / "w", "WRITE_SIZE",
                 [("__amd_rocclr_copyBuffer", write_cal), (k, 500.0), (k, 500.0), (k, 500.0)])
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), workload=workload)
    t = json.load(open(cfg["traffic_file"]))
    assert t["fetch"]["factor"] == pytest.approx(2.0) and t["write"]["factor"] == pytest.approx(1.0)
    assert t["fetch"]["dispatches"] == 3 and t["write"]["dispatches"] == 3
    assert t["fetch"]["bytes_per_launch"] == pytest.approx(2.0 * 2000.0 * 1024)
    assert t["write"]["bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(2.0 * 2000.0 * 1024 + 500.0 * 1024)
    # reported while the kernel sources are the ones hashed, else not at all
    assert bench.measured_traffic(workload) == pytest.approx(t["bytes_per_launch"])
    t["source_sha256"] = "0" * 64
    json.dump(t, open(cfg["traffic_file"], "w"))
    assert bench.measured_traffic(workload) is None
