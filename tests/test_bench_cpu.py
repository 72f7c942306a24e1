"""Host-side checks of the benchmark driver (no GPU): the one-GPU contract, the traffic
table's keying by kernel code, and the algorithmic byte counts it reports against."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_code_hash_ignores_comments_only():
    a = "int f(int x) {\n  // a comment\n  return x + 1;  /* trailing */\n}\n"
    b = "/* header\n   block */\nint f(int x) {\n\n  return x + 1;\n}\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_traffic_lookup_by_path_and_code():
    # every entry of the table names the launch shape it was counted on
    for paths in bench.TRAFFIC.values():
        for entry in paths.values():
            assert entry["bytes_per_iteration"] > 0 and isinstance(entry["launch"], dict)
    assert bench._traffic_for("0000000000000000", {"support_columns": 0}) == (None, None)
    # a count applies to the launch shape it was taken on only
    for kh, paths in bench.TRAFFIC.items():
        for path, entry in paths.items():
            shape = dict(entry["launch"])
            shape.setdefault("support_columns", 1 if "pruned" in path else 0)
            if path.startswith("resident"):
                shape.setdefault("resident_groups", 1)
            assert bench._traffic_for(kh, shape) == (entry["bytes_per_iteration"], entry["launch"])
            other = dict(shape)
            key = next(iter(entry["launch"]))
            other[key] = -1
            assert bench._traffic_for(kh, other) == (None, None)
    kh = bench._kernel_hash(True)
    if kh in bench.TRAFFIC and "resident_pruned" in bench.TRAFFIC[kh]:
        # the cooperative solve moves less than one dense FISTA iteration's 36 B per point
        assert bench.TRAFFIC[kh]["resident_pruned"]["bytes_per_iteration"] < 36 * 256 * 256


@pytest.mark.parametrize("solver,bytes_per_point", [("ista", 28), ("fista", 36), ("admm", 44)])
def test_algorithmic_bytes(solver, bytes_per_point):
    # complex64 grids: ISTA reads c, mu b, Omega and writes c (8+8+4+8); FISTA also reads
    # c_{t-1} (+8); ADMM reads z, v, w, the multiplier and writes z, v (8*5+4)
    assert bench.ALGO_BYTES_PER_POINT[solver] == bytes_per_point
