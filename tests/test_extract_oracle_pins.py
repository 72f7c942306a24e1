"""Pins of the harmonic / direction extraction oracle.

Local maxima are checked against scipy's 3 x 3 maximum filter (a separate implementation of
the same neighbourhood test) on grids without ties, the tie rule on planted ties, the
refinement against the closed form of a two-cell split, the direction inversion by a round
trip through the steering model of eq. (2), and the whole chain (oracle FISTA, then
extraction) by recovering the harmonics of a synthetic scene near its ground truth.
"""
import numpy as np
import pytest
from scipy.ndimage import maximum_filter

from oracle import bccb_oracle as O
from oracle import extract_oracle as X
from paper_2509_13592_amd import scenes as S


def _grid(rng, L2, L1, density=0.05):
    c = np.zeros((L2, L1), dtype=np.complex64)
    n = max(1, int(density * L1 * L2))
    idx = rng.choice(L1 * L2, n, replace=False)
    c.reshape(-1)[idx] = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    return c


@pytest.mark.parametrize("wrap", [True, False])
@pytest.mark.parametrize("shape", [(16, 16), (12, 20), (32, 8)])
def test_local_maxima_match_maximum_filter(wrap, shape):
    rng = np.random.default_rng(shape[0] * 7 + shape[1] + (1 if wrap else 0))
    c = _grid(rng, *shape, density=0.3)
    m = X.mag2_fp32(c)
    thr = np.float32(0.05)
    mode = "wrap" if wrap else "constant"
    mf = maximum_filter(m, size=3, mode=mode, cval=-1.0)
    want = set(np.flatnonzero(((m == mf) & (m > thr)).reshape(-1)).tolist())
    got = {i for _, i in X.local_maxima(c, thr, wrap)}
    assert got == want and len(got) > 0


def test_tie_rule_and_threshold():
    c = np.zeros((8, 8), dtype=np.complex64)
    c[3, 3] = 1.0
    c[3, 4] = 1.0          # equal neighbour with a larger index: (3, 3) wins
    c[6, 1] = 0.5j
    peaks = X.local_maxima(c, 0.0, wrap=True)
    assert sorted(i for _, i in peaks) == [3 + 3 * 8, 1 + 6 * 8]
    assert X.local_maxima(c, 0.25, wrap=True) == [(1.0, 3 + 3 * 8)]   # |0.5j|^2 = 0.25 is not above 0.25


def test_wrap_across_the_grid_edge():
    c = np.zeros((8, 8), dtype=np.complex64)
    c[0, 0] = 0.9
    c[7, 7] = 1.0          # diagonal neighbour of (0, 0) on the wrapped grid
    assert [i for _, i in X.local_maxima(c, 0.0, wrap=True)] == [63]
    assert sorted(i for _, i in X.local_maxima(c, 0.0, wrap=False)) == [0, 63]


def test_refinement_of_a_two_cell_split():
    """A target split over grid points l and l + 1 with magnitudes a and b lands at offset
    b / (a + b); the amplitude is the sum of the two coefficients."""
    for a, b in ((1.0, 0.0), (0.75, 0.25), (0.6, 0.4)):
        c = np.zeros((16, 16), dtype=np.complex64)
        c[5, 7] = a * np.exp(0.3j)
        c[5, 8] = b * np.exp(-1.1j)
        o1, o2, amp = X.refine(c, 7 + 5 * 16, wrap=True)
        assert abs(o1 - b / (a + b)) <= 1e-7 and o2 == 0.0
        assert abs(amp - complex(c[5, 7] + c[5, 8])) <= 1e-7


def test_direction_round_trip_through_eq2():
    rng = np.random.default_rng(3)
    for g1, g2 in ((0.5, 0.5), (0.4, 0.25)):
        for _ in range(200):
            phi = rng.uniform(-np.pi, np.pi)
            theta = rng.uniform(0.0, np.pi / 2)
            f1 = g1 * np.cos(phi) * np.sin(theta)
            f2 = g2 * np.sin(phi) * np.sin(theta)
            p, t = X.direction(f1, f2, g1, g2)
            assert abs(t - theta) <= 1e-7 * max(1.0, 1.0 / max(np.cos(theta), 1e-3))
            if theta > 1e-6:
                assert abs(np.angle(np.exp(1j * (p - phi)))) <= 1e-9 / np.sin(theta)
    assert np.isnan(X.direction(0.45, 0.3, 0.5, 0.5)[1])   # (0.9^2 + 0.6^2) > 1: not a direction


def test_match_recovers_a_permutation():
    truth = np.array([[0.1, 0.2], [-0.3, 0.05], [0.49, -0.49]])
    est = truth[[2, 0, 1]] + 1e-3
    est[0] = [-0.495, 0.495]          # wraps onto truth[2]
    pairs, d = X.match(est, truth)
    assert sorted(pairs) == [(0, 2), (1, 0), (2, 1)]
    assert abs(max(d) - 0.015) <= 1e-12      # |-0.495 - 0.49| = 0.985 wraps to 0.015


def test_chain_recovers_scene_harmonics():
    """Oracle FISTA on a 30 dB scene of well-separated directions, then extraction: every
    target is found within one grid cell, and the directions follow (a target this close to
    the horizon, sin(theta) > 0.95, may be estimated just outside the visible region)."""
    sc = S.angle_scene(0.5, 0.5, 12, 12, 72, 64, 64, K=3, snr_db=30.0, seed=(8, 1, 0), modulus=(0.8, 1.0),
                       min_sep=0.15)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=False)
    c = P.fista(600).reshape(sc.L2, sc.L1).astype(np.complex64)
    peaks = X.extract(c, 3, 0.0)
    est = np.array([[p["f1"], p["f2"]] for p in peaks])
    pairs, d = X.match(est, sc.freqs)
    assert len(pairs) == 3 and max(d) <= 1.0 / 64, d
    for i, j in pairs:
        phi_t, theta_t = sc.meta["angles"][j]
        assert abs(np.angle(np.exp(1j * (peaks[i]["phi"] - phi_t)))) <= 0.05
        if np.sin(theta_t) < 0.95:
            assert abs(peaks[i]["theta"] - theta_t) <= 0.05
