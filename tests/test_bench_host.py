"""Host logic of bench.py (no GPU): the one-GPU guard, the flop count of
the definition, the source and launch-shape check on the stored profile
figures, and the default workload."""
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


def test_profile_figures_are_dropped_once_the_kernel_or_its_shape_changes(tmp_path):
    src = os.path.join(ROOT, "paper_2304_11399_amd", "csrc")
    dst = tmp_path / "paper_2304_11399_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, f), dst / f)
    (tmp_path / "profiles").mkdir()
    shape = {"waves": 2, "item_order": 3, "dense": 0}
    rec = {"workload": "w", "kernel": "k", "shape": shape,
           "source_sha256": bench.kernel_sources_sha(str(tmp_path)),
           "traffic_bytes_per_launch": 123.0}
    json.dump(rec, open(tmp_path / "profiles" / "w_traffic.json", "w"))
    root = str(tmp_path)
    assert bench.measured_profile("w", "k", shape, root)["traffic_bytes_per_launch"] == 123.0
    # another launch shape, another kernel, or a missing record: no figure
    assert bench.measured_profile("w", "k", dict(shape, item_order=1), root) is None
    assert bench.measured_profile("w", "k2", shape, root) is None
    assert bench.measured_profile("no_such_workload", "k", shape, root) is None
    # any kernel source edited since the profile: no figure
    with open(dst / "search.h", "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_profile("w", "k", shape, root) is None


def test_the_default_workload_is_the_binary16_polish_line():
    args = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = args
    assert a.workload == "crs_diff"
    from synth import WORKLOADS
    wl = WORKLOADS["crs_diff"]
    assert wl["store"] == "f16" and wl["de"]["polish_steps"] == 10
    kinds = {v[0] for v in bench.variants_for("crs_diff", dict(wl, name="crs_diff"))}
    assert {"ens_f16_polish", "ens_f16", "ens_f32", "plain_f32"} <= kinds
