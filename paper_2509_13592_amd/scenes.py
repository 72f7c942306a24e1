"""Seeded synthetic single-snapshot scenes for the sparse planar array problem.

This module only draws inputs: an array mask on the half-wavelength grid, target
harmonics and amplitudes, and the noisy snapshot y_s received on the sparse array
(the signal model of eqs. (1)-(3) and (6) of Sec. II-A).  It holds none of the
recovery method's arithmetic (no dictionary, no Gram, no FFT), so both the FP64
oracle and the HIP path can take its outputs as plain inputs.

Conventions
-----------
* mask: uint8 array of shape [M2][M1]; mask[m2, m1] = 1 if the URA element at
  (m1*lambda/2, m2*lambda/2) is kept (the indicator 1_s of Sec. III-A).
* y: complex64 vector of length M = mask.sum(), sensors ordered by increasing
  m1 + m2*M1 (the row order of the subsampling matrix Psi, eq. (6)).
* Harmonics f = (f1, f2) in [-1/2, 1/2)^2; a target contributes
  c_k * exp(-j*2*pi*(m1*f1 + m2*f2)) at element (m1, m2) (eq. (2)).
* SNR = 10*log10(mean_m |y_clean[m]|^2 / sigma^2) with complex Gaussian noise
  CN(0, sigma^2), i.e. real and imaginary parts each N(0, sigma^2/2).

Every scene is drawn from numpy.random.default_rng(SeedSequence([cfg, split, idx]))
in a fixed order: geometry choices -> mask -> K -> frequencies -> amplitude
moduli -> phases -> noise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene",
    "make_scene",
    "tiny_scene",
    "paper_scale_scene",
    "batched_scene",
    "large_admm_scene",
    "learned_scene",
    "learned_fixed_mask",
    "custom_scene",
    "spaced_scene",
    "angle_scene",
    "coefficient_grids",
    "paper_sweep_trials",
    "CONFIG_ITERS",
]

# Solver iteration counts and rho for the five workloads.
CONFIG_ITERS = {1: 200, 2: 500, 3: 300, 4: 300, 5: 16}
CONFIG_RHO = {2: 1.0, 4: 0.5}
TAU_FRACTION = 0.1  # tau = 0.1 * max|A^H y|, computed by whoever consumes the scene


@dataclass
class Scene:
    mask: np.ndarray          # uint8 [M2][M1]
    L1: int
    L2: int
    y: np.ndarray             # complex64 [M]
    freqs: np.ndarray         # float64 [K][2]  (f1, f2)
    amps: np.ndarray          # complex128 [K]
    sigma2: float
    snr_db: float
    cfg: int = 0
    split: int = 0
    idx: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def M1(self) -> int:
        return int(self.mask.shape[1])

    @property
    def M2(self) -> int:
        return int(self.mask.shape[0])

    @property
    def M(self) -> int:
        return int(self.mask.sum())

    def sensors(self) -> np.ndarray:
        """(m1, m2) of each kept element in increasing m1 + m2*M1 order, int64 [M][2]."""
        m2, m1 = np.nonzero(self.mask)  # row-major scan = increasing m1 + m2*M1
        return np.stack([m1, m2], axis=1).astype(np.int64)


def _rng(cfg: int, split: int, idx: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, split, idx]))


def _random_mask(rng: np.random.Generator, M1: int, M2: int, M: int,
                 keep_corners: bool = False) -> np.ndarray:
    mask = np.zeros(M1 * M2, dtype=np.uint8)
    if keep_corners:
        corners = np.array([0, M1 - 1, (M2 - 1) * M1, M2 * M1 - 1])
        mask[corners] = 1
        rest = np.setdiff1d(np.arange(M1 * M2), corners)
        pick = rng.choice(rest, size=M - 4, replace=False)
        mask[pick] = 1
    else:
        pick = rng.choice(M1 * M2, size=M, replace=False)
        mask[pick] = 1
    return mask.reshape(M2, M1)


def _snapshot(rng: np.random.Generator, mask: np.ndarray, K: int, modulus,
              snr_db: float, gammas=None, freqs=None):
    """Draw K targets and the noisy sparse-array snapshot (eqs. (1)-(3), (6)).

    gammas = (gamma1, gamma2): element spacings in wavelengths; the harmonics are then drawn
    from [-gamma1, gamma1) x [-gamma2, gamma2) (Sec. II-A) instead of [-1/2, 1/2)^2.
    freqs: [K][2] harmonics given by the caller (nothing drawn for them)."""
    if freqs is not None:
        freqs = np.asarray(freqs, dtype=np.float64).reshape(K, 2)
    elif gammas is None:
        freqs = rng.uniform(-0.5, 0.5, size=(K, 2))  # f = omega / (2 pi), omega ~ U[-pi, pi)
    else:
        g = np.asarray(gammas, dtype=np.float64)
        freqs = rng.uniform(-g, g, size=(K, 2))
    if modulus is None:
        mod = np.ones(K)
    else:
        mod = rng.uniform(modulus[0], modulus[1], size=K)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=K)
    amps = mod * np.exp(1j * phase)
    m2, m1 = np.nonzero(mask)
    arg = np.outer(m1, freqs[:, 0]) + np.outer(m2, freqs[:, 1])  # [M][K]
    y_clean = np.exp(-2j * np.pi * arg) @ amps
    sigma2 = float(np.mean(np.abs(y_clean) ** 2) / (10.0 ** (snr_db / 10.0)))
    noise = np.sqrt(sigma2 / 2.0) * (rng.standard_normal(len(m1))
                                     + 1j * rng.standard_normal(len(m1)))
    y = (y_clean + noise).astype(np.complex64)
    return y, freqs, amps, sigma2


def custom_scene(M1: int, M2: int, M: int, L1: int, L2: int, K: int, snr_db: float,
                 seed=(0, 0, 0), modulus=None, keep_corners: bool = False,
                 mask: np.ndarray | None = None) -> Scene:
    """A scene of arbitrary geometry (used by tests for ragged and edge shapes)."""
    rng = _rng(*seed)
    if mask is None:
        mask = _random_mask(rng, M1, M2, M, keep_corners)
    else:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, modulus, snr_db)
    return Scene(mask, L1, L2, y, freqs, amps, sigma2, snr_db, cfg=seed[0],
                 split=seed[1], idx=seed[2])


def spaced_scene(gamma1: float, gamma2: float, M1: int, M2: int, M: int, L1: int, L2: int, K: int,
                 snr_db: float, seed=(7, 0, 0), modulus=(0.5, 1.0)) -> Scene:
    """An array with element spacing (gamma1 lambda, gamma2 lambda): M of the M1 x M2 URA
    elements kept (corners included, aperture preserved), K targets with harmonics uniform in
    [-gamma_i, gamma_i), |c_k| ~ U[modulus].  The snapshot model is that of eq. (3):
    element (m1, m2) sees exp(-j 2 pi (m1 f1 + m2 f2))."""
    rng = _rng(*seed)
    mask = _random_mask(rng, M1, M2, M, keep_corners=M >= 4 and M1 > 1 and M2 > 1)
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, modulus, snr_db, gammas=(gamma1, gamma2))
    return Scene(mask, L1, L2, y, freqs, amps, sigma2, snr_db, cfg=seed[0], split=seed[1], idx=seed[2],
                 meta={"gamma": (gamma1, gamma2)})


def angle_scene(gamma1: float, gamma2: float, M1: int, M2: int, M: int, L1: int, L2: int, K: int,
                snr_db: float, seed=(8, 0, 0), modulus=(0.5, 1.0), min_sep: float = 0.0) -> Scene:
    """Targets drawn as directions: azimuth phi ~ U[-pi, pi), elevation theta ~ U[0, pi/2)
    (the ranges of Sec. II-A), each mapped to its harmonics by the steering model of eq. (2),
    (f1, f2) = (gamma1 cos(phi) sin(theta), gamma2 sin(phi) sin(theta)).  min_sep > 0 redraws
    a direction whose harmonics lie closer than min_sep (max-norm, in cycles) to an earlier
    target's.  meta['angles'] holds the [K][2] (phi, theta) drawn."""
    rng = _rng(*seed)
    mask = _random_mask(rng, M1, M2, M, keep_corners=M >= 4 and M1 > 1 and M2 > 1)
    angles = np.empty((K, 2))
    freqs = np.empty((K, 2))
    k = 0
    while k < K:
        phi = rng.uniform(-np.pi, np.pi)
        theta = rng.uniform(0.0, np.pi / 2)
        f = np.array([gamma1 * np.cos(phi) * np.sin(theta), gamma2 * np.sin(phi) * np.sin(theta)])
        if k and min_sep > 0 and np.abs(freqs[:k] - f).max(axis=1).min() < min_sep:
            continue
        angles[k] = (phi, theta)
        freqs[k] = f
        k += 1
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, modulus, snr_db, freqs=freqs)
    return Scene(mask, L1, L2, y, freqs, amps, sigma2, snr_db, cfg=seed[0], split=seed[1], idx=seed[2],
                 meta={"gamma": (gamma1, gamma2), "angles": angles})


def coefficient_grids(seed, batch: int, L1: int, L2: int, n_blobs: int = 6, n_scatter: int = 40) -> np.ndarray:
    """complex64 [batch][L2][L1] grids shaped like sparse recovered coefficient grids: each holds
    n_blobs 3 x 3 blobs (a random centre value, neighbours scaled by U[0, 0.8]) and n_scatter
    isolated small entries (|c| <= 0.3), all at random positions (wrapping at the edges)."""
    rng = _rng(*seed)
    out = np.zeros((batch, L2, L1), dtype=np.complex64)
    for b in range(batch):
        g = out[b]
        for _ in range(n_blobs):
            c1, c2 = int(rng.integers(L1)), int(rng.integers(L2))
            centre = rng.uniform(0.5, 1.0) * np.exp(1j * rng.uniform(0, 2 * np.pi))
            for d2 in (-1, 0, 1):
                for d1 in (-1, 0, 1):
                    f = 1.0 if d1 == 0 and d2 == 0 else rng.uniform(0.0, 0.8)
                    g[(c2 + d2) % L2, (c1 + d1) % L1] = centre * f * np.exp(1j * rng.uniform(-0.3, 0.3))
        pos = rng.choice(L1 * L2, size=min(n_scatter, L1 * L2), replace=False)
        g.reshape(-1)[pos] = (0.3 * rng.uniform(0, 1, len(pos)) * np.exp(1j * rng.uniform(0, 2 * np.pi, len(pos))))
    return out


def tiny_scene(idx: int = 0) -> Scene:
    """8x8 URA, 32 of 64 kept, L1 = L2 = 32, K = 3 unit-modulus targets, 20 dB."""
    rng = _rng(1, 0, idx)
    mask = _random_mask(rng, 8, 8, 32)
    K = 3
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, None, 20.0)
    return Scene(mask, 32, 32, y, freqs, amps, sigma2, 20.0, 1, 0, idx)


def paper_sweep_scene(L1: int, idx: int = 0) -> Scene:
    """The geometry of the paper's runtime sweep (Sec. III-C): a 51 x 16 URA with 40 elements
    kept, the aperture preserved (corner elements kept), L2 = 32, L1 = the sweep value,
    K ~ U{1..10} unit-modulus targets, 15 dB."""
    rng = _rng(6, L1, idx)
    mask = _random_mask(rng, 51, 16, 40, keep_corners=True)
    K = int(rng.integers(1, 11))
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, None, 15.0)
    return Scene(mask, L1, 32, y, freqs, amps, sigma2, 15.0, 6, L1, idx)


def paper_sweep_trials(L1: int, n: int = 10) -> list:
    """n trials of the paper's runtime sweep geometry (Sec. III-C) on ONE array: the 51 x 16 URA
    with 40 elements kept including the corners (drawn once for the whole sweep), L2 = 32,
    L1 = the sweep value; each trial draws its own K ~ U{1..10} unit-modulus targets, harmonics
    and 15 dB noise."""
    mask = _random_mask(_rng(6, 0, 999), 51, 16, 40, keep_corners=True)
    out = []
    for idx in range(n):
        rng = _rng(6, 1000 + L1, idx)
        K = int(rng.integers(1, 11))
        y, freqs, amps, sigma2 = _snapshot(rng, mask, K, None, 15.0)
        out.append(Scene(mask, L1, 32, y, freqs, amps, sigma2, 15.0, 6, 1000 + L1, idx))
    return out


def paper_scale_scene(idx: int = 0) -> Scene:
    """16x16 URA, 64 of 256 kept, L1 = L2 = 256, K = 5, |c_k| ~ U[0.5, 1], 20 dB."""
    rng = _rng(2, 0, idx)
    mask = _random_mask(rng, 16, 16, 64)
    K = 5
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, (0.5, 1.0), 20.0)
    return Scene(mask, 256, 256, y, freqs, amps, sigma2, 20.0, 2, 0, idx)


def batched_scene(idx: int) -> Scene:
    """One of the 4096 uneven scenes: 16x16 or 32x32 array, 25-50 % kept,
    L1 = L2 in {64, 128, 256}, K ~ U{1..8}, SNR ~ U[10, 30] dB."""
    rng = _rng(3, 0, idx)
    side = 16 if rng.uniform() < 0.5 else 32
    density = rng.uniform(0.25, 0.5)
    Lg = int(rng.choice([64, 128, 256]))
    snr = float(rng.uniform(10.0, 30.0))
    M = max(1, int(round(density * side * side)))
    mask = _random_mask(rng, side, side, M)
    K = int(rng.integers(1, 9))
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, (0.5, 1.0), snr)
    return Scene(mask, Lg, Lg, y, freqs, amps, sigma2, snr, 3, 0, idx,
                 meta={"density": density})


def large_admm_scene(idx: int = 0) -> Scene:
    """32x32 URA, 256 of 1024 kept, L1 = L2 = 1024, K = 10 unit-modulus, 15 dB."""
    rng = _rng(4, 0, idx)
    mask = _random_mask(rng, 32, 32, 256)
    K = 10
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, None, 15.0)
    return Scene(mask, 1024, 1024, y, freqs, amps, sigma2, 15.0, 4, 0, idx)


def learned_fixed_mask() -> np.ndarray:
    """The one array geometry of the learned workload (16x16 URA, 64 of 256)."""
    return _random_mask(_rng(5, 0, 0), 16, 16, 64)


def learned_scene(split: int, idx: int, mask: np.ndarray | None = None) -> Scene:
    """Learned-solver scene: fixed mask, K ~ U{1..8}, SNR ~ U[10, 30] dB,
    |c_k| ~ U[0.5, 1].  split 0 = training, split 1 = held-out evaluation."""
    if mask is None:
        mask = learned_fixed_mask()
    rng = _rng(5, 1 + split, idx)
    snr = float(rng.uniform(10.0, 30.0))
    K = int(rng.integers(1, 9))
    y, freqs, amps, sigma2 = _snapshot(rng, mask, K, (0.5, 1.0), snr)
    return Scene(mask, 256, 256, y, freqs, amps, sigma2, snr, 5, split, idx)


def learned_batch(split: int, start: int, count: int, mask: np.ndarray | None = None):
    """Snapshots of `count` learned-workload scenes stacked as complex64 [count][M]."""
    if mask is None:
        mask = learned_fixed_mask()
    ys = np.stack([learned_scene(split, start + i, mask).y for i in range(count)])
    return mask, ys


def make_scene(cfg: int, idx: int = 0, split: int = 0) -> Scene:
    if cfg == 1:
        return tiny_scene(idx)
    if cfg == 2:
        return paper_scale_scene(idx)
    if cfg == 3:
        return batched_scene(idx)
    if cfg == 4:
        return large_admm_scene(idx)
    if cfg == 5:
        return learned_scene(split, idx)
    raise ValueError(f"unknown workload {cfg}")
