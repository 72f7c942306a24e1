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
        for entries in paths.values():
            for entry in entries:
                assert entry["bytes_per_iteration"] > 0 and isinstance(entry["launch"], dict)
    assert bench._traffic_for("0000000000000000", {"support_columns": 0}) == (None, None)
    # a count applies to the launch shape it was taken on only
    for kh, paths in bench.TRAFFIC.items():
        for path, entries in paths.items():
            for entry in entries:
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
    for entry in bench.TRAFFIC.get(kh, {}).get("resident_pruned", []):
        # the cooperative solve moves less than one dense FISTA iteration's 36 B per point
        assert entry["bytes_per_iteration"] < 36 * 256 * 256


@pytest.mark.parametrize("solver,bytes_per_point", [("ista", 28), ("fista", 36), ("admm", 44)])
def test_algorithmic_bytes(solver, bytes_per_point):
    # complex64 grids: ISTA reads c, mu b, Omega and writes c (8+8+4+8); FISTA also reads
    # c_{t-1} (+8); ADMM reads z, v, w, the multiplier and writes z, v (8*5+4)
    assert bench.ALGO_BYTES_PER_POINT[solver] == bytes_per_point


def test_pruned_byte_model():
    """Algorithmic bytes of one pruned FISTA iteration: kept spectra moved four times, iterate
    rows as slot rows (count + index + value) while sparse and as dense rows otherwise."""
    import numpy as np
    L1 = L2 = 256
    ncs = 16
    empty = bench.pruned_bytes_per_iteration(L1, L2, ncs, np.zeros(L2, int))
    assert empty == 32 * ncs * L2 + 3 * 4 * L2
    one = np.zeros(L2, int)
    one[3] = 5
    assert bench.pruned_bytes_per_iteration(L1, L2, ncs, one) == empty + 3 * 50
    dense = np.full(L2, L1, int)
    assert bench.pruned_bytes_per_iteration(L1, L2, ncs, dense) == 32 * ncs * L2 + 3 * L2 * (4 + 8 * L1)
    # a row just over L1/8 nonzeros is stored dense
    edge = np.zeros(L2, int)
    edge[0] = L1 // 8 + 1
    assert bench.pruned_bytes_per_iteration(L1, L2, ncs, edge) == empty + 3 * 8 * L1
    # never more than the full passes move per point (48 B with the row-spectral exchange)
    assert bench.pruned_bytes_per_iteration(L1, L2, ncs, dense) <= 48 * L1 * L2 * 2


def test_batch_fraction_is_a_fraction():
    """A rate at exactly the HBM peak gives frac 1; the bytes model is stated on the line."""
    r = bench._batch_roofline(bench.HBM_PEAK_GBS * 1e9 * 2.0, 2.0)
    assert abs(r["frac_hbm_peak"] - 1.0) < 1e-9 and "bytes_model" in r
    r = bench._batch_roofline(1e9, 1.0)
    assert 0 < r["frac_hbm_peak"] < 1


def test_counted_tables_are_well_formed():
    # the counted full-pass bytes and the persistent launch's VALU count name the launch
    # shape / workload they were taken on, and each applies only to its own source version
    for kh, shapes in bench.FULL_BATCH_TRAFFIC.items():
        assert len(kh) == 16
        for shape, bpp in shapes.items():
            assert len(shape) == 4 and all(isinstance(v, int) and v > 0 for v in shape)
            # the two full passes move at least the dense iteration's 36 B per point
            assert 36 <= bpp <= 64
    for kh, entry in bench.PERSISTENT_VALU.items():
        assert len(kh) == 16
        scenes, n, iters = entry["workload"]
        assert scenes > 0 and n in (32, 64, 128, 256) and iters > 0
        assert entry["valu_per_scene_iteration"] > 0
    assert bench._persistent_hash() != bench._kernel_hash()
