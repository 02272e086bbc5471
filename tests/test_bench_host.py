"""Host logic of bench.py (no GPU): the one-GPU guard, the flop count of
the definition and the source check on the stored HBM-traffic figure."""
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_flops_per_pair_counts_the_definition():
    # CRS: 11 for the traveltime, 6 per window sample, 1 for 1 - f
    assert bench.flops_per_pair(3, 7) == 11 + 6 * 7 + 1
    # CMP: the moveout is one product
    assert bench.flops_per_pair(1, 5) == 7 + 6 * 5 + 1


def test_traffic_figure_is_dropped_once_the_kernel_sources_change(tmp_path, monkeypatch):
    import hashlib
    src = os.path.join(ROOT, "paper_2304_11399_amd", "csrc")
    dst = tmp_path / "paper_2304_11399_amd" / "csrc"
    dst.mkdir(parents=True)
    h = hashlib.sha256()
    for f in ("device.h", "kernels.hip"):
        shutil.copy(os.path.join(src, f), dst / f)
        h.update(open(dst / f, "rb").read())
    (tmp_path / "profiles").mkdir()
    rec = {"workload": "w", "kernel": "k", "source_sha256": h.hexdigest(),
           "traffic_bytes_per_launch": 123.0}
    json.dump(rec, open(tmp_path / "profiles" / "w_traffic.json", "w"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w")["traffic_bytes_per_launch"] == 123.0
    with open(dst / "kernels.hip", "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_traffic("w") is None
    assert bench.measured_traffic("no_such_workload") is None
