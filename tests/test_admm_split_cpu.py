"""The pruned ADMM forms (the cooperative kernel and the pruned passes) run eqs. (13)-(15) with
the scaled dual split as v_t = u_t + IDFT2(Psi_t), u_t = z_{t-1} - z_t and Psi on the support
bins of Omega.  This checks on the CPU, in FP64, that the rearranged iteration produces the
same z and x as the oracle's ADMM written in the paper's order: the rearrangement is exact, so
the two agree to rounding (a dropped term, a wrong sign or a shifted index in it would not).
"""
import numpy as np
import pytest

from oracle import bccb_oracle as O
from paper_2509_13592_amd import scenes as S


def _soft(x, k):
    a = np.abs(x)
    return np.where(a > k, x * (1.0 - k / np.maximum(a, 1e-300)), 0.0)


def split_admm(P, rho, iters):
    """ADMM through the split form, with unnormalised DFT2 / IDFT2 (IDFT2(DFT2(x)) = L x)."""
    L1, L2 = P.op.L1, P.op.L2
    L = L1 * L2
    e0 = np.zeros(L, complex)
    e0[0] = 1.0
    omega = np.real(np.fft.fft2(P.op.gram(e0).reshape(L2, L1)))   # the Gram's eigenvalues
    sup = np.abs(omega) > 1e-9 * np.abs(omega).max()
    b = P.b.reshape(L2, L1)
    s = np.where(sup, np.fft.fft2(b) / L, 0.0)                      # DFT2(b) = L S, on the support only
    dft2 = np.fft.fft2
    idft2 = lambda v: np.fft.ifft2(v) * L
    d = 1.0 / (omega + rho)
    kappa = P.tau / rho
    z = np.zeros((L2, L1), complex)
    zp = z.copy()
    psi = np.zeros((L2, L1), complex)
    x = z
    for _ in range(iters):
        y = dft2(2 * z - zp)                                            # DFT2(z_t - u_t)
        vp = np.where(sup, (s - rho * psi - omega * y / L) * d, 0.0)   # V'
        psi = psi + vp
        x = (2 * z - zp) + idft2(vp)                                    # x_{t+1}
        zn = _soft(z + idft2(psi), kappa)                               # z_{t+1} = S(x_{t+1} + v_t)
        zp, z = z, zn
    return z.reshape(-1), x.reshape(-1)


@pytest.mark.parametrize("idx,rho,iters", [(0, 1.0, 130), (3, 4.0, 60), (0, 40.0, 60)])
def test_split_dual_admm_is_the_paper_update(idx, rho, iters):
    sc = S.tiny_scene(idx)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    zr, xr = P.admm(rho, iters)
    z, x = split_admm(P, rho, iters)
    ez = np.linalg.norm(z - zr) / max(np.linalg.norm(zr), 1e-300)
    ex = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    assert np.count_nonzero(zr) > 0   # the threshold is exercised: some elements are kept
    assert ez <= 1e-9 and ex <= 1e-9, (ez, ex)


def test_split_dual_admm_rectangular_grid():
    sc = S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(12, 0, 0))
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    zr, xr = P.admm(2.0, 40)
    z, x = split_admm(P, 2.0, 40)
    assert np.linalg.norm(z - zr) <= 1e-9 * max(np.linalg.norm(zr), 1e-300)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
