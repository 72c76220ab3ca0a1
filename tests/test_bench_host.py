"""Host logic of bench.py (no GPU): a committed counter record counts as the
bench line's `traffic` only for the kernel source and the workload it was
taken on."""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(mod, "ROOT", str(tmp_path))
    return mod


def _record(tmp_path, src_hash, alg=None, total=1.5e9):
    rec = {"kernel": "k", "source": "src.hip", "source_sha256_16": src_hash, "bytes_per_launch": total}
    if alg is not None:
        rec["algorithmic_bytes_per_launch"] = alg
    (tmp_path / "profiles" / "rec.json").write_text(json.dumps(rec))


def test_traffic_needs_the_same_source(bench, tmp_path):
    src = tmp_path / "src.hip"
    src.write_text("kernel v1\n")
    _record(tmp_path, bench._src_hash(str(src)))
    assert bench._traffic(str(src), "rec.json") == 1.5e9
    src.write_text("kernel v2\n")  # the source changed after the counters were taken
    assert bench._traffic(str(src), "rec.json") is None


def test_traffic_needs_the_same_workload(bench, tmp_path):
    src = tmp_path / "src.hip"
    src.write_text("kernel\n")
    h = bench._src_hash(str(src))
    _record(tmp_path, h, alg=1.0e9)
    assert bench._traffic(str(src), "rec.json", 1.0e9) == 1.5e9
    assert bench._traffic(str(src), "rec.json", 1.009e9) == 1.5e9  # within 1%
    assert bench._traffic(str(src), "rec.json", 1.02e9) is None  # another workload
    _record(tmp_path, h)  # no workload recorded: only a source check is possible
    assert bench._traffic(str(src), "rec.json") == 1.5e9
    assert bench._traffic(str(src), "rec.json", 1.0e9) is None


def test_traffic_missing_record(bench, tmp_path):
    src = tmp_path / "src.hip"
    src.write_text("kernel\n")
    assert bench._traffic(str(src), "absent.json") is None
