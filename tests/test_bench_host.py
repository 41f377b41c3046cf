"""Host-side logic of bench.py (no GPU): the one-GPU rule and the lookup of
the committed HBM counter summary that fills `roofline.traffic`."""
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
    val, why = bench.measured_traffic("block_dot")
    if why == "kernels changed since the counters were taken":
        pytest.skip("the counter summary was taken on other kernel code (traffic is null)")
    assert why is None
    assert val == pytest.approx(c["fetch_bytes"] + c["write_bytes"])
    assert c["fetch_bytes"] > 0 and c["write_bytes"] >= 0
    assert bench.measured_traffic("no_such_class")[0] is None


def test_traffic_is_withheld_for_other_kernel_code(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    val, why = bench.measured_traffic("block_dot")
    assert val is None and "changed" in why
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("block_dot") == (None, "no counter summary")
