"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte model of the
roofline, and the rule that counter-measured traffic is reported only for the sources it was
taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("cls, s, f, want", [
    ("postsmooth16", 4, 8, 16.5),   # read x, b, q, 1/8 coarse correction; write x
    ("presmooth16", 4, 8, 8.5),     # read b; write x and 1/8 restricted residual
    ("apply16", 4, 8, 16.0),
    ("update", 4, 8, 12.0),
    ("update", 8, 8, 24.0),
    ("resid64", 4, 8, 20.0),
    ("ir", 4, 8, 24.0),             # read p (8), d and the last direction; write p (8)
    ("correct", 4, 8, 56.0),
    ("correct", 4, 4, 32.0),
])
def test_algorithmic_bytes_per_cell(cls, s, f, want):
    assert bench.alg_bytes_per_cell(cls, s, f) == pytest.approx(want)


def test_forcing_bytes_scale_with_the_body_fraction():
    assert bench.alg_bytes_per_cell("force", 4, 8, body=0.0) == 8
    assert bench.alg_bytes_per_cell("force", 4, 8, body=1.0) == 8 + 48


def test_latency_classes_have_no_byte_model():
    assert bench.alg_bytes_per_cell("coarse", 4, 8) is None
    assert bench.alg_bytes_per_cell("finalize", 4, 8) is None


def test_level_cells():
    n = 33_554_432
    assert bench.level_cells("presmooth16", n, 16) == n
    assert bench.level_cells("postsmooth8", n, 16) == n / 8
    assert bench.level_cells("presmooth2", n, 16) == n / 512
    assert bench.level_cells("resid64", n, 16) == n


def test_traffic_only_for_the_sources_it_was_taken_on(monkeypatch):
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    d = json.load(open(path))
    key = next(iter(d["kernels"]))
    workload, precision, cls = key.split("/")
    monkeypatch.setattr(bench, "source_hash", lambda: d["source_sha256"])
    assert bench.measured_traffic(cls, workload, precision) == d["kernels"][key]["hbm_bytes_per_launch"]
    assert bench.measured_traffic("no_such_class", workload, precision) is None
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(cls, workload, precision) is None
