"""Host-side checks of bench.py's measurement bookkeeping (no GPU): the HBM
traffic it reports comes from the committed rocprofv3 record only while the
kernel code and the timed tile shape match that record."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

RECORD = os.path.join(ROOT, "profiles", "stage_kernel_mhd3d_uneven4096_traffic.json")


def record():
    with open(RECORD) as f:
        return json.load(f)


def test_comment_edits_keep_the_hash_and_code_edits_change_it():
    src = "int f(int x) {\n  // a comment\n  return x + 1; /* another */\n}\n"
    assert bench.strip_comments(src) == bench.strip_comments(src.replace("a comment", "edited"))
    assert bench.strip_comments(src) != bench.strip_comments(src.replace("x + 1", "x + 2"))

    def reader(edit):
        def read(path):
            with open(os.path.join(ROOT, path)) as f:
                s = f.read()
            return edit(s) if path.endswith("kernels.hip") else s
        return read

    h0 = bench.kernel_source_hash()
    assert bench.kernel_source_hash(reader(lambda s: s + "\n// trailing comment\n")) == h0
    assert bench.kernel_source_hash(reader(lambda s: s + "\nstatic int unused_probe;\n")) != h0


def test_traffic_is_reported_for_recorded_shapes_of_the_current_code():
    rec = record()
    if rec["kernel_source_hash"] != bench.kernel_source_hash():
        pytest.skip("the traffic record predates the current kernel code")
    assert bench.measured_traffic(rec["variant"], rec["form"]) == rec["bytes_per_stage"]
    for name, v in rec["variants"].items():   # the per-class pass covers every shape
        assert bench.measured_traffic(name, "per_class") == v["bytes_per_stage"]
    if rec["form"] == "single":
        others = [n for n in rec["variants"] if n != rec["variant"]]
        assert all(bench.measured_traffic(n, "single") is None for n in others)
    assert bench.measured_traffic("no-such-tile-shape", rec["form"]) is None


def test_traffic_is_withheld_when_the_code_changes(monkeypatch):
    rec = record()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda read=None: "0" * 16)
    assert bench.measured_traffic(rec["variant"], rec["form"]) is None


def test_record_is_calibrated_and_consistent():
    rec = record()
    kib = 1024.0
    assert rec["copy_probe"]["bytes"] / kib / rec["copy_probe"]["fetch_size_kib"] == pytest.approx(rec["read_factor"])
    assert rec["copy_probe"]["bytes"] / kib / rec["copy_probe"]["write_size_kib"] == pytest.approx(rec["write_factor"])
    # a stage is launches_per_stage dispatches: one per block-size class, or one
    assert rec["launches_per_stage"] == {"per_class": 3, "single": 1}[rec["form"]]
    total = rec["launches_per_stage"] * (rec["fetch_size_kib_per_dispatch"] * kib * rec["read_factor"]
                                         + rec["write_size_kib_per_dispatch"] * kib * rec["write_factor"])
    assert total == pytest.approx(rec["bytes_per_stage"], rel=1e-6)
    # algorithmic bytes: 17 state passes x 8 variables x 8 bytes per cell and step, over 5 stages
    assert rec["algorithmic_bytes_per_stage"] == pytest.approx(
        bench.BYTES_PER_CELL_STEP_MHD3D / bench.STAGES * 25160192)
    # every shape in the per-class autotuning pass of the same run
    for v in rec["variants"].values():
        assert v["bytes_per_stage"] > rec["algorithmic_bytes_per_stage"]


def test_other_lists_traffic_is_reported_per_shape():
    rec = record()
    if rec["kernel_source_hash"] != bench.kernel_source_hash():
        pytest.skip("the traffic record predates the current kernel code")
    assert set(rec["others"]) == set(bench.FORWARD_LEGS)
    for leg, o in rec["others"].items():
        kib = 1024.0
        assert o["copy_probe"]["bytes"] / kib / o["copy_probe"]["fetch_size_kib"] == pytest.approx(o["read_factor"])
        assert o["copy_probe"]["bytes"] / kib / o["copy_probe"]["write_size_kib"] == pytest.approx(o["write_factor"])
        for name, v in o["variants"].items():
            assert bench.measured_traffic_other(leg, name) == v["bytes_per_stage"]
            # one launch per stage: bytes = calibrated FETCH + WRITE of one dispatch
            total = v["fetch_size_kib_per_dispatch"] * kib * o["read_factor"] + \
                v["write_size_kib_per_dispatch"] * kib * o["write_factor"]
            assert total == pytest.approx(v["bytes_per_stage"], rel=1e-6)
            assert v["bytes_per_stage"] > 0.9 * v["algorithmic_bytes_per_stage"]
        assert bench.measured_traffic_other(leg, "no-such-tile-shape") is None
