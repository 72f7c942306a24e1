"""GPU parity of bccb_extract_peaks (harmonics and directions from coefficient grids) with the
extraction oracle, on seeded synthetic grids consumed by both sides: the selected grid indices
and their order are integer decisions taken in FP32 on both sides and must agree exactly; the
refined harmonics within 1e-6 cycles (FP32 weights against FP64), amplitudes within 1e-5
relative, directions within 1e-4 rad where the inversion is well conditioned; and on a scene
solved on the GPU the chain recovers the generator's harmonics.
"""
import numpy as np
import pytest

from oracle import bccb_oracle as O
from oracle import extract_oracle as X
from paper_2509_13592_amd import scenes as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2509_13592_amd.bccb")


def _compare(rec, ref, what):
    assert rec is not None, what
    assert [int(r) for r in rec["index"]] == [p["index"] for p in ref], what
    for r, p in zip(rec, ref):
        assert r["mag2"] == np.float32(p["mag2"]), what
        for k in ("f1", "f2"):
            d = abs(float(r[k]) - p[k])
            assert min(d, 1.0 - d) <= 1e-6, (what, k, float(r[k]), p[k])
        amp = complex(r["amp_re"], r["amp_im"])
        assert abs(amp - p["amp"]) <= 1e-5 * max(1.0, abs(p["amp"])), what
        assert abs(np.angle(np.exp(1j * (float(r["phi"]) - p["phi"])))) <= 1e-4, what
        if np.isnan(p["theta"]) or np.isnan(r["theta"]):
            s2 = (p["f1"] / 0.5) ** 2 + (p["f2"] / 0.5) ** 2
            assert np.isnan(p["theta"]) == np.isnan(r["theta"]) or abs(s2 - 1.0) <= 1e-5, what
        elif np.cos(p["theta"]) > 1e-2:
            assert abs(float(r["theta"]) - p["theta"]) <= 1e-4, what


@pytest.mark.parametrize("L1,L2,batch", [(64, 64, 3), (256, 256, 4), (32, 128, 2)])
def test_extract_matches_oracle_half_spacing(L1, L2, batch):
    grids = S.coefficient_grids((9, L1, L2), batch, L1, L2)
    mask = np.ones((4, 4), dtype=np.uint8)
    plan = B.Plan(mask, L1, L2)
    c = B.to_device(grids)
    for K, thr in ((8, 0.0), (3, 0.05), (64, 0.01)):
        recs = plan.extract_peaks(c, K, thr)
        for b in range(batch):
            ref = X.extract(grids[b], K, thr)
            print(f"case extract {L1}x{L2} grid {b} K={K} thr={thr}: {len(ref)} peaks", flush=True)
            _compare(recs[b], ref, (L1, L2, b, K))
    plan.close()


def test_extract_spaced_grid_no_wrap():
    L1, L2, g1, g2 = 48, 40, 0.4, 0.25
    grids = S.coefficient_grids((9, 1, 2), 3, L1, L2)
    sc = S.spaced_scene(g1, g2, 6, 5, 17, L1, L2, K=2, snr_db=20.0)
    plan = B.SpacedPlan(sc.mask, L1, L2, g1, g2)
    recs = plan.extract_peaks(B.to_device(grids), 10, 0.0)
    for b in range(3):
        ref = X.extract(grids[b], 10, 0.0, g1, g2)
        assert [int(r) for r in recs[b]["index"]] == [p["index"] for p in ref]
        for r, p in zip(recs[b], ref):
            assert abs(float(r["f1"]) - p["f1"]) <= 1e-6 and abs(float(r["f2"]) - p["f2"]) <= 1e-6
    plan.close()


def test_extract_ties_threshold_and_overflow():
    plan = B.Plan(np.ones((2, 2), dtype=np.uint8), 16, 16)
    g = np.zeros((16, 16), dtype=np.complex64)
    g[3, 3] = g[3, 4] = 1.0          # equal neighbours: the smaller index is the maximum
    g[9, 9] = 0.5j
    g[0, 0] = 0.7
    g[15, 15] = 0.7                  # equal across the wrapped corner: index 0 wins
    rec = plan.extract_peaks(B.to_device(g), 10, 0.0)[0]
    assert [int(i) for i in rec["index"]] == [p["index"] for p in X.extract(g, 10, 0.0)] == [51, 0, 153]
    rec = plan.extract_peaks(B.to_device(g), 10, 0.25)[0]   # 0.25 = |0.5j|^2 is not above it
    assert [int(i) for i in rec["index"]] == [51, 0]
    rec = plan.extract_peaks(B.to_device(g), 1, 0.0)[0]
    assert [int(i) for i in rec["index"]] == [51]
    plan.close()
    # a grid with 128 x 128 / 4 isolated maxima (> 4096) is refused for that grid only
    plan = B.Plan(np.ones((2, 2), dtype=np.uint8), 256, 256)
    many = np.zeros((2, 256, 256), dtype=np.complex64)
    rng = np.random.default_rng(1)
    many[0, ::2, ::2] = (0.5 + rng.uniform(0, 1, (128, 128))).astype(np.complex64)
    many[1, 10, 20] = 1.0
    recs = plan.extract_peaks(B.to_device(many), 4, 0.0)
    assert recs[0] is None and [int(i) for i in recs[1]["index"]] == [20 + 10 * 256]
    plan.close()


def test_chain_on_gpu_recovers_harmonics():
    """GPU FISTA then GPU extraction on a 30 dB scene of separated directions: every target
    within one grid cell of its harmonic tuple."""
    sc = S.angle_scene(0.5, 0.5, 16, 16, 96, 128, 128, K=4, snr_db=30.0, seed=(8, 2, 0), modulus=(0.8, 1.0),
                       min_sep=0.12)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=False)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    c = plan.fista(B.to_device(sc.y), P.tau, 800)
    rec = plan.extract_peaks(c, 4, 0.0)[0]
    est = np.stack([rec["f1"], rec["f2"]], axis=1).astype(float)
    pairs, d = X.match(est, sc.freqs)
    print(f"case chain: distances {np.round(d, 5)} (cell {1 / 128:.4f})", flush=True)
    assert len(pairs) == 4 and max(d) <= 1.0 / 128
    plan.close()


def test_extract_odd_sized_grid():
    """A half-spacing grid of 45 x 27 points (an odd count: the kernel reads single points, not
    pairs), wrapping at the edges."""
    L1, L2 = 45, 27
    grids = S.coefficient_grids((9, 2, 3), 3, L1, L2)
    sc = S.spaced_scene(0.5, 0.5, 7, 5, 20, L1, L2, K=2, snr_db=20.0)
    plan = B.SpacedPlan(sc.mask, L1, L2, 0.5, 0.5)
    recs = plan.extract_peaks(B.to_device(grids), 12, 0.0)
    for b in range(3):
        _compare(recs[b], X.extract(grids[b], 12, 0.0), (L1, L2, b))
    plan.close()


def test_extract_more_peaks_than_threads():
    """600 isolated maxima and max_peaks = 400 (more peaks than the selecting workgroup has
    threads): the 400 strongest, in order, as the oracle lists them."""
    L = 128
    rng = np.random.default_rng(21)
    g = np.zeros((L, L), dtype=np.complex64)
    pos = rng.choice((L // 2) * (L // 2), 600, replace=False)
    r2, r1 = 2 * (pos // (L // 2)), 2 * (pos % (L // 2))
    g[r2, r1] = (rng.uniform(0.1, 1.0, 600) * np.exp(1j * rng.uniform(0, 2 * np.pi, 600))).astype(np.complex64)
    plan = B.Plan(np.ones((2, 2), dtype=np.uint8), L, L)
    rec = plan.extract_peaks(B.to_device(g), 400, 0.0)[0]
    _compare(rec, X.extract(g, 400, 0.0), "many")
    assert len(rec) == 400
    plan.close()
