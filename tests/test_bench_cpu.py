"""Host logic of bench.py: committed counter summaries are used only while the
kernel source and the launch shape match the ones they were taken on (else
the figure is reported as null), and more than one GPU is refused.  No GPU
here."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary(tmp_path, sha, launch):
    path = tmp_path / "summary.json"
    path.write_text(json.dumps({"kernel_source_sha256": sha,
                                "pair_mixed_n16384": {"kernel_source_sha256": sha,
                                                      "launch": launch,
                                                      "bytes_per_launch": 123.0}}))
    return str(path)


def test_profile_value_needs_matching_source_and_launch(tmp_path):
    sha = bench.kernel_source_sha()
    launch = {"symmetric": 2, "sym_variant": 7}
    good = _summary(tmp_path, sha, launch)
    assert bench.profile_value(good, "pair_mixed_n16384", dict(launch, i_per_lane=4),
                               "bytes_per_launch") == 123.0
    # another launch shape, another kernel key, another source, a missing file
    assert bench.profile_value(good, "pair_mixed_n16384", {"symmetric": 2, "sym_variant": 6},
                               "bytes_per_launch") is None
    assert bench.profile_value(good, "pair_fp64_n16384", launch, "bytes_per_launch") is None
    stale = _summary(tmp_path, "0" * 64, launch)
    assert bench.profile_value(stale, "pair_mixed_n16384", launch, "bytes_per_launch") is None
    assert bench.profile_value(str(tmp_path / "absent.json"), "pair_mixed_n16384", launch,
                               "bytes_per_launch") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
