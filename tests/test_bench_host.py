"""Host-side checks of the benchmark's contract (no GPU): the one-GPU guard,
the flop counts the roofline uses, and that measured HBM traffic is reported
only for the sources and workloads it was measured on."""
import argparse
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _args(**kw):
    a = dict(config="headline", tile=16, storage="f32", oit=False, alpha_cut=0.0)
    a.update(kw)
    return argparse.Namespace(**a)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_flops_per_pair():
    assert bench.flops_per_pair("raster_fwd", False) == 20
    assert bench.flops_per_pair("raster_bwd", False) == 48
    assert bench.flops_per_pair("raster_fwd", True) == 23
    assert bench.flops_per_pair("raster_bwd", True) == 56


def test_traffic_only_for_the_measured_sources_and_workloads():
    for t in bench.TRAFFIC:
        args = _args(**t["workload"])
        if bench._source_sha(t["source"]) != t["source_sha"]:
            assert bench.traffic_bytes(t["kernel"], args) is None
            continue
        got = bench.traffic_bytes(t["kernel"], args)
        want = t["fetch_kib"] * 1024 / t["fetch_factor"] + t["write_kib"] * 1024 / t["write_factor"]
        assert got == pytest.approx(want, rel=1e-12)
        # another tile, storage or kernel has no measurement
        assert bench.traffic_bytes(t["kernel"], argparse.Namespace(**{**vars(args), "tile": 8})) is None
        assert bench.traffic_bytes(t["kernel"], argparse.Namespace(**{**vars(args), "storage": "bf16"})) is None
        assert bench.traffic_bytes("raster_fwd", args) is None


def test_algorithmic_bytes_scale_with_the_work():
    a = bench.algorithmic_bytes(1000, 4096, "f32", 5000)
    b = bench.algorithmic_bytes(2000, 4096, "f32", 5000)
    assert all(v > 0 for v in a.values())
    assert b["project"] > a["project"] and b["raster_bwd"] > a["raster_bwd"]
    assert bench.algorithmic_bytes(1000, 4096, "bf16", 5000)["project"] < a["project"]
