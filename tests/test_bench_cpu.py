"""Host logic of bench.py (CPU only): the single-GPU refusal, the
per-workload smoothing table, and the traffic records of profiles/."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_every_workload_has_valid_smoothing():
    assert set(bench.SWEEPS) == set(bench.WORKLOADS)
    for name, (nu1, nu2, coarse) in bench.SWEEPS.items():
        assert 0 <= nu1 <= 8 and 0 <= nu2 <= 8 and nu1 + nu2 > 0, name
        c1, c2 = divmod(coarse, 16)
        assert coarse == 0 or (0 <= c1 <= 8 and 0 <= c2 <= 8 and c1 + c2 > 0), name


@pytest.mark.parametrize("workload", ["bubble2d_1024", "wall3d_256", "collapse3d_512",
                                      "state2d_1024", "axi2d_1024"])
def test_traffic_records(workload):
    """Each committed record names the roofline kernel class and the
    commands that made it; bench.py uses it only while the kernel sources
    hash as they did when the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path) as fh:
        rec = json.load(fh)
    assert rec["kernel_class"] == bench.ROOFLINE_KERNEL
    assert rec["hbm_bytes_per_launch"] > 0
    assert all("rocprofv3 --pmc" in c for c in rec["commands"])
    got = bench.traffic_from_profile(workload, bench.ROOFLINE_KERNEL, 1)
    if rec["source_hash"] == bench.kernel_source_hash():
        assert got == rec["hbm_bytes_per_launch"]
    else:
        assert got is None
    assert bench.traffic_from_profile(workload, "not_a_class", 1) is None


def test_small_workload_shapes():
    p = bench.make_problem("explicit_64")
    assert p.n[:2] == (64, 64) and p.dim == 2
    with pytest.raises(SystemExit):
        bench.make_problem("explicit_64", stiff=True)
