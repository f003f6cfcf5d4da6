"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the counter
record's link to the kernel source, and the measured-traffic lookup."""
import json
import os
import re
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
    assert r.stdout == ""


def test_source_digest_ignores_comments_only():
    d = bench.kernel_source_digest()
    assert len(d) == 64 and d == bench.kernel_source_digest()


def _algorithmic(key):
    """Algorithmic HBM bytes per launch of a recorded workload/form key: 20
    state values read and written per cell, 4 bytes each in the
    float32-state form, 8 in float64."""
    import re

    from paper_2411_15001_amd import cases

    bpc = 160 if key.endswith("_fp32") else 320
    if key.startswith("batch256"):
        return sum(int(n) ** 2 for n in cases.batch_sides(256, seed=0)) * bpc
    m = re.match(r"(blast|rarefaction)(\d+)_", key)
    return int(m.group(2)) ** 2 * bpc


def _record():
    with open(bench.PMC_FILE) as f:
        return json.load(f)


def test_traffic_lookup_matches_launch_shape():
    rec = _record()
    if rec.get("source_sha256") != bench.kernel_source_digest():
        pytest.skip("the step kernel changed since its counters were recorded")
    if not os.path.exists(os.path.join(ROOT, "paper_2411_15001_amd", "libvlbm.so")):
        pytest.skip("library not built")
    for key, entry in rec.items():
        if not isinstance(entry, dict) or "launch" not in entry:
            continue
        launch = entry["launch"]
        got = bench.traffic_for(key, launch)
        assert got == entry["bytes_per_launch"], key
        # the measured bytes lie at most 15% above the algorithmic ones (the
        # re-read halo rows and columns) and not below them
        assert entry["algorithmic_bytes"] == _algorithmic(key), key
        ratio = got / _algorithmic(key)
        assert 1.0 <= ratio < 1.15, (key, ratio)
        # another strip height has other halo re-reads: no figure
        other = [launch[0] * 2] + list(launch[1:])
        assert bench.traffic_for(key, other) is None
        # missing trailing launch values read as 0
        assert bench.traffic_for(key, launch[:2]) == (got if all(v == 0 for v in launch[2:]) else None)
    assert bench.traffic_for("no_such_workload", [64, 4]) is None


def test_other_workloads_summarise_and_keep_going(monkeypatch):
    """The default run's `also`: each other workload runs without its CPU
    baseline and without printing its own line, is summarised (forms and
    roofline kept), and a failing one is recorded in place of its figures
    without losing the others."""
    import bench

    seen = []

    def fake(name):
        def run(b):
            seen.append((name, b.no_cpu, b.emit, getattr(b, "n", None), getattr(b, "forms", None)))
            if name == "batch":
                raise RuntimeError("no device")
            line = {"config": {"workload": name}, "metric": "m", "value": 1.0, "unit": "GLUPS",
                    "ms_per_step": 2.0, "steps": 5, "roofline": {"frac": 0.5}}
            if name == "rarefaction":
                line["forms"] = {"fp64": {"value": 1.0, "ms_per_step": 2.0, "launch": [256, 1, 4, 0],
                                          "roofline": {"frac": 0.5}, "diag": {}}}
            return line
        return run

    monkeypatch.setattr(bench, "bench_rarefaction", fake("rarefaction"))
    monkeypatch.setattr(bench, "bench_batch", fake("batch"))
    monkeypatch.setattr(bench, "bench_adjoint", fake("adjoint"))
    import sys

    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.headline_only is False
    out = bench.other_workloads(a)
    assert set(out) == {"rarefaction8192_lmp", "batch256", "adjoint512"}
    assert "error" in out["batch256"] and "no device" in out["batch256"]["error"]
    assert out["rarefaction8192_lmp"]["forms"]["fp64"]["launch"] == [256, 1, 4, 0]
    assert "diag" not in out["rarefaction8192_lmp"]["forms"]["fp64"]
    assert all(no_cpu and not emit for _, no_cpu, emit, _, _ in seen)
    assert ("rarefaction", True, False, 8192, "fp64,fp32") in seen
    assert a.no_cpu is False  # the caller's options are not changed


def test_traffic_records_use_the_committed_launch_shapes():
    """Every counter record was taken in the launch shape that the committed
    autotune cache gives its workload, so the default benchmark run, which
    reads its shapes from that cache, finds a record (a shape changed in one
    file and not the other would leave `traffic` null)."""
    with open(os.path.join(ROOT, "paper_2411_15001_amd", "autotune_cache.json")) as f:
        cache = json.load(f)
    # record key -> (instances, nx, precision, limiter set, boundary conditions)
    want = {"blast8192_fp32": ("1", "8192", "1", "9", "00"), "blast8192_fp64": ("1", "8192", "0", "9", "00"),
            "rarefaction8192_fp32": ("1", "8192", "1", "11", "11"),
            "rarefaction8192_fp64": ("1", "8192", "0", "11", "11"),
            "rarefaction8192_rlmp_fp32": ("1", "8192", "1", "13", "11"),
            "rarefaction8192_rlmp_fp64": ("1", "8192", "0", "13", "11"),
            "rarefaction2048_fp64": ("1", "2048", "0", "11", "11"), "batch256_fp32": ("256", None, "1", "9", "11")}
    rec = _record()
    for key, (n, nx, prec, lims, bc) in want.items():
        assert key in rec, key
        hits = []
        for ck, shape in cache.items():
            m = re.match(r"n(\d+)_nx(\d+)_ny\d+_cells\d+_p(\d)_lim(\d+)_o2_bc(\d\d)_s0_b0_h", ck)
            if m and m.group(1) == n and (nx is None or m.group(2) == nx) and m.group(3) == prec \
                    and m.group(4) == lims and m.group(5) == bc:
                hits.append(shape)
        assert len(hits) == 1, (key, hits)
        assert list(hits[0]) == list(rec[key]["launch"]), (key, hits[0], rec[key]["launch"])
