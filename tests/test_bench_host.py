"""Host logic of bench.py (no GPU): the one-GPU contract, the workload
table and the traffic figure's tie to the kernel source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU only" in r.stderr


@pytest.mark.parametrize("name,n", [("large", 1), ("bench", 1), ("tiny", 1), ("sweep", 32), ("paper", 1),
                                    ("paperscan", 11)])
def test_workloads(name, n):
    import bench
    desc, cfgs = bench.workload(name)
    assert len(cfgs) == n and desc
    if name == "large":
        assert cfgs[0]["N"] == 16384 and cfgs[0]["n_load"] == 16384000


def test_unknown_workload():
    import bench
    with pytest.raises(SystemExit):
        bench.workload("nope")


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    import hashlib
    import bench
    src = hashlib.sha256(open(bench.KERNEL_SOURCE, "rb").read()).hexdigest()
    if src in open(bench.TRAFFIC_PROFILE).read():
        assert bench.measured_traffic() > 0
    else:
        assert bench.measured_traffic() is None
    other = tmp_path / "k.hip"
    other.write_text("// not the profiled kernel\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(other))
    assert bench.measured_traffic() is None
