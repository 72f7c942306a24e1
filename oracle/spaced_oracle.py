"""Plain FP64 (complex128) reference for harmonic grids at a general element spacing.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Sec. II-A places element (m1, m2) at (m1 gamma1 lambda, m2 gamma2 lambda); the harmonic of
dimension i then lies in [-gamma_i, gamma_i), and Sec. III-A samples it on the uniform grid
f_{i,l} = -gamma_i + l (2 gamma_i / L_i), l = 0..L_i-1 (eq. (16)).  On that grid the Gram
D_i^H D_i is Toeplitz; it is circulant only at gamma_i = 1/2, the case the rest of the oracle
(bccb_oracle) is written for.  D_s^H D_s is the masked Kronecker sum of eq. (17), here with
Toeplitz factors, i.e. block Toeplitz with Toeplitz blocks.

This module writes the subdictionaries of eq. (5) on that grid for a rational gamma_i = p/q
(the phase f_{i,l} m = p (2l - L_i) m / (q L_i) is taken from an exact integer residue) and any
grid length L_i >= 1, and wraps them in bccb_oracle.Operator, whose products
D_s c = (D_2 C D_1^T) at the kept elements and D_s^H y = D_2^H Y conj(D_1) (eq. (4)) use only
these factors -- no FFT.  The LASSO pieces (step size, soft threshold, ISTA, FISTA, ADMM,
objective, KKT residual) are bccb_oracle's, called with this operator; the shifted inverse of
the ADMM step is rebuilt here from this operator's own Gram.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import bccb_oracle as O

HALF = Fraction(1, 2)


def spacing(gamma) -> Fraction:
    """gamma as an exact fraction in (0, 1] (floats are read as the nearest p/q, q <= 2^20)."""
    g = gamma if isinstance(gamma, Fraction) else Fraction(gamma).limit_denominator(1 << 20)
    if not (0 < g <= 1):
        raise ValueError("element spacing gamma must lie in (0, 1]")
    return g


def harmonic_grid(L: int, gamma) -> np.ndarray:
    """f_l = -gamma + l (2 gamma / L), l = 0..L-1 (eq. (16))."""
    g = float(spacing(gamma))
    return -g + np.arange(L) * (2.0 * g / L)


def subdictionary(M: int, L: int, gamma) -> np.ndarray:
    """D_i(m, l) = exp(-j 2 pi f_l m), m < M, l < L, on the grid of eq. (16) (eq. (5)).

    With gamma = p/q, f_l m = p (2l - L) m / (q L) exactly, so the phase is the residue
    (p (2l - L) m) mod (q L) divided by q L."""
    g = spacing(gamma)
    p, q = g.numerator, g.denominator
    m = np.arange(M, dtype=np.int64)[:, None]
    l = np.arange(L, dtype=np.int64)[None, :]
    k = (p * (2 * l - L) * m) % (q * L)
    return np.exp(-1j * O.TWO_PI * k / (q * L))


class Operator(O.Operator):
    """D_s, D_s^H and the Gram on the grid of spacing (gamma1, gamma2) and any L1, L2."""

    def __init__(self, mask: np.ndarray, L1: int, L2: int, gamma1=HALF, gamma2=HALF):
        super().__init__(mask, L1, L2)
        self.gamma1, self.gamma2 = spacing(gamma1), spacing(gamma2)
        self.D1 = subdictionary(self.M1, self.L1, self.gamma1)
        self.D2 = subdictionary(self.M2, self.L2, self.gamma2)


def sparse_dictionary(op: Operator) -> np.ndarray:
    """D_s = Psi (D_2 kron D_1), complex128 [M][L1 L2] (eqs. (4), (7)); column l1 + l2 L1."""
    s = op.s
    rows = op.D2[s[:, 1], :][:, :, None] * op.D1[s[:, 0], :][:, None, :]
    return rows.reshape(op.M, op.L)


def gram_dense(op: Operator) -> np.ndarray:
    """Explicit G = D_s^H D_s, complex128 [L][L] (left-hand side of eq. (17))."""
    Ds = sparse_dictionary(op)
    return Ds.conj().T @ Ds


class ShiftedInverse:
    """x -> (G + rho I)^-1 x for the ADMM c-update (eq. (13)) on the spaced grid: Cholesky of
    the explicit G + rho I for small L, else the Woodbury form
    (1/rho)(I - D_s^H (rho I_M + D_s D_s^H)^-1 D_s) through the operator."""

    def __init__(self, op: Operator, rho: float, dense_limit: int = 4096):
        self.op = op
        self.rho = float(rho)
        self.dense = op.L <= dense_limit
        if self.dense:
            self.chol = np.linalg.cholesky(gram_dense(op) + rho * np.eye(op.L))
        else:
            self.small = np.linalg.inv(rho * np.eye(op.M) + op.outer_gram())

    def __call__(self, x):
        x = np.asarray(x, dtype=np.complex128)
        if self.dense:
            t = np.linalg.solve(self.chol, x)
            return np.linalg.solve(self.chol.conj().T, t)
        return (x - self.op.adjoint(self.small @ self.op.forward(x))) / self.rho


class Problem:
    """One scene's LASSO in FP64 on the spaced grid: D_s, b = D_s^H y_s, mu, tau."""

    def __init__(self, mask, L1, L2, y, gamma1=HALF, gamma2=HALF, tau=None, tau_fraction=0.1, dense=None):
        self.op = Operator(mask, L1, L2, gamma1, gamma2)
        self.y = np.asarray(y, dtype=np.complex64).astype(np.complex128)
        self.b = self.op.adjoint(self.y)
        self.mu = O.step_size(self.op)
        if tau is None:
            tau = np.float32(tau_fraction * np.abs(self.b).max())
        self.tau = float(np.float32(tau))
        if dense is None:
            dense = self.op.L <= 4096
        self.G = gram_dense(self.op) if dense else None

    def apply_G(self, x):
        return self.G @ x if self.G is not None else self.op.gram(x)

    def ista(self, iters, c0=None):
        return O.ista(self.apply_G, self.b, self.mu, self.tau, iters, c0)

    def fista(self, iters, c0=None):
        return O.fista(self.apply_G, self.b, self.mu, self.tau, iters, c0)

    def admm(self, rho, iters):
        return O.admm(ShiftedInverse(self.op, rho), self.b, rho, self.tau, iters)

    def objective(self, c):
        return O.objective(self.op, self.y, c, self.tau)

    def kkt(self, c):
        return O.kkt_residual(self.op, self.b, c, self.tau)
