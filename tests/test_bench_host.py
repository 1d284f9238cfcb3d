"""Host-side pieces of bench.py that need no GPU: the one-GPU guard, the
algorithmic byte count behind roofline.achieved, and the rule that a stored
HBM-traffic record is used only while the kernel sources are unchanged."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2506_09242_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr, (r.returncode, r.stderr)
    assert r.stdout.strip() == ""


def test_algorithmic_bytes():
    # headline: every node fluid, one model, no walls -> untagged, no tag bytes
    tags = inputs.all_fluid(8, 8, 8, inputs.TAG_SMAG)
    b, fluid = bench.alg_bytes_per_launch(tags, 27, 4, tagged=False)
    assert fluid == 512 and b == 512 * 2 * 27 * 4
    # 512^3 D3Q27 FP32: the figure the profiles and roofline.achieved use
    assert 512 ** 3 * 2 * 27 * 4 == 28_991_029_248
    # walled cavity: fluid nodes move 2 Q s bytes, every node one tag byte
    t = inputs.cavity_tags(16)
    b, fluid = bench.alg_bytes_per_launch(t, 19, 2, tagged=True)
    assert fluid == 14 ** 3 and b == 14 ** 3 * 2 * 19 * 2 + 16 ** 3
    # solid nodes cost only their tag byte
    t = np.zeros((4, 4, 4), np.uint8)
    t[0, 0, 0] = inputs.TAG_TRT
    assert bench.alg_bytes_per_launch(t, 19, 8) == (2 * 19 * 8 + 64, 1)


def test_traffic_records_follow_the_kernel_sources(monkeypatch):
    p = os.path.join(ROOT, "profiles", "traffic_tgv512_d3q27_smag_f32.json")
    rec = json.load(open(p))
    assert rec["alg_bytes_per_launch"] == 28_991_029_248
    # the committed record belongs to the committed kernel sources
    assert rec["source_hash"] == bench.source_hash()
    assert bench.stored_traffic("tgv512_d3q27_smag", "f32") == rec["bytes_per_launch"]
    # once the sources change, the record is not used
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.stored_traffic("tgv512_d3q27_smag", "f32") is None
    assert bench.stored_traffic("no_such_workload", "f32") is None
