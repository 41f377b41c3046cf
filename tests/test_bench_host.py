"""Host-side logic of bench.py (no GPU): the one-GPU rule and the lookup of
the committed HBM counter summary that fills `roofline.traffic` (only for
the kernel code and the workload the counters were taken on)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv,
                       capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, **env))
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_comes_from_the_committed_summary_of_these_kernels():
    with open(bench.TRAFFIC_FILE) as f:
        tr = json.load(f)
    c = tr["classes"]["block_dot"]
    val, why = bench.measured_traffic("block_dot", "porous256_ir")
    if why == "kernels changed since the counters were taken":
        pytest.skip("the counter summary was taken on other kernel code (traffic is null)")
    assert why is None
    assert val == pytest.approx(c["fetch_bytes"] + c["write_bytes"])
    assert c["fetch_bytes"] > 0 and c["write_bytes"] >= 0
    assert bench.measured_traffic("no_such_class", "porous256_ir")[0] is None


def test_traffic_is_withheld_for_other_kernel_code(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    val, why = bench.measured_traffic("block_dot", "porous256_ir")
    assert val is None and "changed" in why
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("block_dot", "porous256_ir") == (None, "no counter summary")


def _args(argv):
    return bench.make_parser().parse_args(argv)


@pytest.mark.parametrize("argv", [["--n", "128"], ["--shape", "256", "256", "32"], ["--k", "10"],
                                  ["--m", "20"], ["--local-solver", "ssor"],
                                  ["--inner-tol", "1e-6"], ["--n-switch", "2"]])
def test_traffic_is_withheld_for_other_workloads(argv):
    a = _args(argv)
    w = bench.counter_workload(a)
    val, why = bench.measured_traffic("block_dot", w)
    assert val is None and "another workload" in why
    assert bench.counter_workload(_args([])) == "porous256_ir"


def test_shape_applies_to_the_default_workload_only():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "serve",
                        "--shape", "64", "64", "32"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "--shape applies to the default workload" in p.stderr
    assert p.stdout == ""
