"""Host logic of bench.py (no GPU): the one-GPU refusal, the error norms of
the reduced forms against FP64, and the HBM-traffic lookup keyed by the
sweep source."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_error_norms():
    """Relative L2 and L-inf over cells active in both runs; mismatching
    classes counted over all cells."""
    torch = pytest.importorskip("torch")
    flags_a = torch.tensor([2, 2, 1, 0, 1], dtype=torch.uint8)
    flags_b = torch.tensor([2, 1, 1, 0, 0], dtype=torch.uint8)
    u_a = torch.tensor([[1.0, 2.0, 2.0, 9.0, 5.0], [0.0, 0.0, 0.0, 9.0, 5.0], [0.0, 0.0, 0.0, 9.0, 5.0]],
                       dtype=torch.float64)
    u_b = u_a.clone()
    u_b[0, 1] = 2.5
    phi_a = torch.tensor([1.0, 1.0, 0.5, 0.0, 0.3], dtype=torch.float64)
    phi_b = phi_a.clone()
    e = bench.errors({"flags": flags_a, "u": u_a, "phi": phi_a}, {"flags": flags_b, "u": u_b, "phi": phi_b})
    assert e["flag_mismatch"] == 2
    # active in both: cells 0, 1, 2
    assert e["u_l2"] == pytest.approx(0.5 / 3.0)
    assert e["u_linf"] == pytest.approx(0.5 / 2.0)
    assert e["phi_l2"] == 0.0 and e["phi_linf"] == 0.0


def test_traffic_lookup(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    d = {"source_hash": "abc", "cells": 1000, "forms": {"fp16s": {"bytes_per_launch": 123.0}}}
    (tmp_path / "profiles" / "sweep_traffic.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "abc")
    assert bench.traffic_for("fp16s", 1000) == 123.0
    assert bench.traffic_for("fp32", 1000) is None
    assert bench.traffic_for("fp16s", 999) is None  # counters of another lattice
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "changed")
    assert bench.traffic_for("fp16s", 1000) is None


def test_committed_counters_match_the_sweep_source():
    """The committed counter summary was taken on the current sweep source, so
    the benchmark line carries the measured traffic."""
    d = json.load(open(os.path.join(ROOT, "profiles", "sweep_traffic.json")))
    assert d["source_hash"] == bench.sweep_source_hash()
    assert d["cells"] == 512 * 320 * 512
    for form in ("fp64", "fp32", "fp16s"):
        assert 1.0 <= d["forms"][form]["ratio_to_algorithmic"] < 1.1
    assert np.isclose(d["calibration"]["write_factor"], 1.0, atol=0.01)
