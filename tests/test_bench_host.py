"""Host logic of bench.py (no GPU): the time-to-eps selection, the product
byte counts and the traffic-file reader."""
import os
import types

import pytest

import bench


def test_time_to_eps_picks_the_smallest_q(monkeypatch):
    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    errs = {0: 2.0, 1: 0.05, 2: 0.004, 3: 0.0031, 4: 0.003}
    calls = []

    def solve_q(q):
        calls.append(q)
        return types.SimpleNamespace(Z=q)

    out = bench.time_to_eps(solve_q, lambda Z: errs[Z], 4)
    assert [r["q"] for r in out["sweep"]] == [0, 1, 2, 3, 4]
    assert out["0.1"]["q"] == 1 and out["0.01"]["q"] == 2
    assert out["0.001"] == "not reached"
    assert calls.count(2) == 4          # one warm-up and three timed solves per q


def test_product_bytes():
    ax, aty = bench.csr_product_bytes(11000, 130000, 1_470_000, 20)
    assert ax == 1_470_000 * 8 + 11001 * 4 + 130000 * 20 * 4 + 11000 * 20 * 4
    assert aty == 1_470_000 * 8 + 130001 * 4 + 11000 * 20 * 4 + 130000 * 20 * 4
    ax, aty = bench.dense_product_bytes(2000, 1000, 10, 8, 8)
    assert ax == aty == 2000 * 1000 * 8 + 1000 * 10 * 8 + 2000 * 10 * 8


def test_traffic_reader_requires_matching_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_traffic.txt").write_text("# c\nsource_sha: abc\ntraffic_bytes_per_launch: 123\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("k", "abc") == 123.0
    assert bench.read_traffic("k", "def") is None
    assert bench.read_traffic("missing", "abc") is None
    assert os.path.exists(prof / "k_traffic.txt")


def test_value_unit_follows_the_ridge():
    # FP32 dense products above the FP32 matrix-core ridge (157.3 TFLOP/s
    # over 8 TB/s: 19.7 flop/B) report TFLOP/s; below it, or in BF16 / FP8,
    # or on CSR, GB/s
    assert bench.value_unit("dense", "f32", 131072, 32768, 256, 4) == "TFLOP/s"   # AI 128
    assert bench.value_unit("dense", "f32", 65536, 16384, 100, 4) == "TFLOP/s"    # AI 50
    assert bench.value_unit("dense", "f32", 8192, 4096, 32, 4) == "GB/s"          # AI 16
    assert bench.value_unit("dense", "f64", 2000, 1000, 10, 8) == "GB/s"          # AI 2.5
    assert bench.value_unit("dense", "fp8", 131072, 32768, 256, 1) == "GB/s"
    assert bench.value_unit("csr", "f32", 11000, 130000, 20, 4) == "GB/s"
    assert bench.rate("TFLOP/s", 1e9, 2e12, 1000.0) == pytest.approx(2.0)
    assert bench.rate("GB/s", 4e9, 1.0, 500.0) == pytest.approx(8.0)
