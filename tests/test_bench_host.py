"""Host-side logic of the benchmark (CPU only): the single-GPU contract, and
the rule that a committed counter summary is used only while the kernel
sources it was taken on are unchanged."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("n", ["2", "8", "0"])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_committed_summaries_name_their_sources(bench):
    """Every kernel summary names its sources and their hash, and gives the
    command that produced it."""
    for path in (bench.TRAFFIC_FILE, bench.COUNTERS_FILE):
        with open(path) as fh:
            doc = json.load(fh)
        assert doc["kernels"]
        assert "rocprofv3" in json.dumps(doc.get("commands", doc.get("command")))
        for name, k in doc["kernels"].items():
            assert k["sources"] and len(k["source_hash"]) == 16, name


def test_current_summary_is_used(bench, tmp_path, monkeypatch):
    """A summary whose hash is that of the current sources is read."""
    for attr in ("TRAFFIC_FILE", "COUNTERS_FILE"):
        with open(getattr(bench, attr)) as fh:
            doc = json.load(fh)
        k = doc["kernels"]["icgn_f32"]
        k["sources"] = list(bench.KERNEL_SOURCES["icgn_f32"])
        k["source_hash"] = bench.kernel_source_hash(k["sources"])
        p = tmp_path / os.path.basename(getattr(bench, attr))
        p.write_text(json.dumps(doc))
        monkeypatch.setattr(bench, attr, str(p))
    assert bench.measured_traffic("icgn_f32") > 0
    assert 0 < bench.measured_issue("icgn_f32", 0.5)["valu_issue_frac"]


def test_stale_summary_is_not_used(bench, tmp_path, monkeypatch):
    """A summary whose source hash differs from the current sources gives
    null traffic and issue fractions."""
    for attr in ("TRAFFIC_FILE", "COUNTERS_FILE"):
        with open(getattr(bench, attr)) as fh:
            doc = json.load(fh)
        doc["kernels"]["icgn_f32"]["source_hash"] = "0" * 16
        p = tmp_path / os.path.basename(getattr(bench, attr))
        p.write_text(json.dumps(doc))
        monkeypatch.setattr(bench, attr, str(p))
    assert bench.measured_traffic("icgn_f32") is None
    assert bench.measured_issue("icgn_f32", 0.5) is None


def test_batched_oracle_extrapolation(bench):
    """The batched oracle sample weights each subset size's per-POI time by
    the 64 pairs' POI counts and divides over the processes (a stand-in pool
    returns a known time per POI and subset size)."""
    import dicgen

    per_poi = {15: 0.004, 21: 0.005, 31: 0.006, 41: 0.008}

    class Pool:
        def map(self, fn, chunks):
            out = []
            for k, idx in chunks:
                sub = dicgen.batch_pair_params(k)[2]
                out.append((per_poi[sub] * len(idx), len(idx), sub))
            return out

    r = bench.oracle_batched_sample(Pool(), 16)
    n_total, t_total = 0, 0.0
    for k in range(64):
        sub = dicgen.batch_pair_params(k)[2]
        n = len(dicgen.poi_grid(512, 512, sub // 2, 8, 6))
        n_total += n
        t_total += n * per_poi[sub]
    assert r["pois"] == 8 * 128 and r["extrapolated_pois"] == n_total
    assert r["pois_per_s"] == pytest.approx(n_total / (t_total / 16), rel=1e-3)
    assert r["seconds_per_poi_by_subset"] == {str(k): v for k, v in per_poi.items()}
