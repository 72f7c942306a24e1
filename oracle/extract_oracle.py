"""Plain reference for turning a recovered coefficient grid into harmonics and directions.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Sec. II-A: the support of the sparse estimate c (eq. (7)) marks the harmonic tuples
(f_{1,l1}, f_{2,l2}) present (column l1 + l2 L1 of D, eq. (4)), and each harmonic tuple
gives a direction through eq. (2): f1 = gamma1 cos(phi) sin(theta), f2 = gamma2 sin(phi)
sin(theta), phi in [-pi, pi), theta in [0, pi/2).

Readings taken here (the paper names the step but not its details):
  * a harmonic is a local maximum of |c| over its 8 grid neighbours whose |c|^2 exceeds a
    threshold; on the half-spacing grid (gamma = 1/2) the grid wraps (f = -1/2 and f = 1/2
    are the same harmonic), on narrower spacings it does not;
  * the comparison is on |c|^2 = re*re + im*im formed in FP32 (each product and the sum
    rounded to FP32), the precision the coefficients come in; equal values are ordered by
    the linear index l1 + l2 L1, the smaller index ranking higher (so of two equal
    neighbours only the one with the smaller index can be a maximum);
  * at most K harmonics are reported, by decreasing |c|^2 (ties: smaller index first);
  * each is refined to the |c|-weighted mean of its 3 x 3 neighbourhood's grid offsets
    (a target between grid points splits its amplitude over the neighbours), the amplitude
    being the sum of the neighbourhood's coefficients;
  * a harmonic pair with (f1/gamma1)^2 + (f2/gamma2)^2 > 1 has no direction (it lies
    outside the visible region of eq. (2)): theta is reported as NaN.
"""
from __future__ import annotations

import numpy as np


def mag2_fp32(c: np.ndarray) -> np.ndarray:
    """|c|^2 formed in FP32: re*re and im*im each rounded, then their sum rounded."""
    c = np.asarray(c, dtype=np.complex64)
    re = c.real.astype(np.float32)
    im = c.imag.astype(np.float32)
    return (re * re).astype(np.float32) + (im * im).astype(np.float32)


def grid_harmonic(l: int, L: int, gamma: float) -> float:
    """f_l = -gamma + l (2 gamma / L) (eq. (16))."""
    return -gamma + l * (2.0 * gamma / L)


def local_maxima(c_grid: np.ndarray, min_mag2: float, wrap: bool) -> list[tuple[float, int]]:
    """(|c|^2, index) of every grid point above the threshold that beats all 8 neighbours,
    written out point by point."""
    L2, L1 = c_grid.shape
    m = mag2_fp32(c_grid)
    thr = np.float32(min_mag2)
    out = []
    for l2 in range(L2):
        for l1 in range(L1):
            v = m[l2, l1]
            if not v > thr:
                continue
            idx = l1 + l2 * L1
            best = True
            for d2 in (-1, 0, 1):
                for d1 in (-1, 0, 1):
                    if d1 == 0 and d2 == 0:
                        continue
                    n1, n2 = l1 + d1, l2 + d2
                    if wrap:
                        n1 %= L1
                        n2 %= L2
                    elif not (0 <= n1 < L1 and 0 <= n2 < L2):
                        continue
                    w = m[n2, n1]
                    nidx = n1 + n2 * L1
                    if w > v or (w == v and nidx < idx):
                        best = False
            if best:
                out.append((float(v), idx))
    return out


def refine(c_grid: np.ndarray, idx: int, wrap: bool) -> tuple[float, float, complex]:
    """|c|-weighted mean grid offset (o1, o2) over the 3 x 3 neighbourhood and the sum of its
    coefficients."""
    L2, L1 = c_grid.shape
    l1, l2 = idx % L1, idx // L1
    sw = s1 = s2 = 0.0
    amp = 0j
    for d2 in (-1, 0, 1):
        for d1 in (-1, 0, 1):
            n1, n2 = l1 + d1, l2 + d2
            if wrap:
                n1 %= L1
                n2 %= L2
            elif not (0 <= n1 < L1 and 0 <= n2 < L2):
                continue
            v = complex(c_grid[n2, n1])
            w = abs(v)
            sw += w
            s1 += w * d1
            s2 += w * d2
            amp += v
    return (s1 / sw, s2 / sw, amp) if sw > 0 else (0.0, 0.0, amp)


def direction(f1: float, f2: float, gamma1: float, gamma2: float) -> tuple[float, float]:
    """(phi, theta) with f1 = gamma1 cos(phi) sin(theta), f2 = gamma2 sin(phi) sin(theta)
    (eq. (2)); theta = NaN outside the visible region."""
    u, v = f1 / gamma1, f2 / gamma2
    s2 = u * u + v * v
    phi = float(np.arctan2(v, u))
    if phi >= np.pi:
        phi -= 2 * np.pi
    theta = float(np.arcsin(np.sqrt(s2))) if s2 <= 1.0 else float("nan")
    return phi, theta


def extract(c_grid: np.ndarray, max_peaks: int, min_mag2: float, gamma1: float = 0.5, gamma2: float = 0.5):
    """Harmonics and directions of a coefficient grid [L2][L1]: a list of dicts with the grid
    index, |c|^2, refined (f1, f2), amplitude and (phi, theta), strongest first."""
    L2, L1 = c_grid.shape
    wrap = gamma1 == 0.5 and gamma2 == 0.5
    peaks = local_maxima(c_grid, min_mag2, wrap)
    peaks.sort(key=lambda t: (-t[0], t[1]))
    out = []
    for mag2, idx in peaks[:max_peaks]:
        l1, l2 = idx % L1, idx // L1
        o1, o2, amp = refine(c_grid, idx, wrap)
        f1 = grid_harmonic(l1, L1, gamma1) + o1 * (2.0 * gamma1 / L1)
        f2 = grid_harmonic(l2, L2, gamma2) + o2 * (2.0 * gamma2 / L2)
        if wrap:
            f1 = (f1 + 0.5) % 1.0 - 0.5
            f2 = (f2 + 0.5) % 1.0 - 0.5
        phi, theta = direction(f1, f2, gamma1, gamma2)
        out.append({"index": idx, "mag2": mag2, "f1": f1, "f2": f2, "amp": amp, "phi": phi, "theta": theta})
    return out


def match(est: np.ndarray, truth: np.ndarray, period: float | None = 1.0):
    """Pairs estimated and true harmonic tuples ([n][2] each) one to one, minimising the sum of
    max-norm distances (wrapped by `period` when given), by the Hungarian assignment
    (scipy's linear_sum_assignment).  Returns (pairs (est index, truth index), distances)."""
    from scipy.optimize import linear_sum_assignment

    est = np.asarray(est, dtype=float).reshape(-1, 2)
    truth = np.asarray(truth, dtype=float).reshape(-1, 2)
    if len(est) == 0 or len(truth) == 0:
        return [], []
    d = np.abs(est[:, None, :] - truth[None, :, :])
    if period is not None:
        d = np.minimum(d, period - d)
    cost = d.max(axis=2)
    r, c = linear_sum_assignment(cost)
    pairs = list(zip(r.tolist(), c.tolist()))
    return pairs, [float(cost[i, j]) for i, j in pairs]
