"""Plain FP64 (complex128) reference for the sparse-array LASSO and its BCCB Gram.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Everything here follows the paper's definitions directly:

* the harmonic grid f_{i,l} = -1/2 + l/L_i (eq. (16) with gamma_i = 1/2);
* the subdictionaries D_i(m, l) = exp(-j 2 pi f_{i,l} m) (eq. (5)) and
  D = D_2 kron D_1 (eq. (4)), the column of (l1, l2) being l1 + l2*L1;
* the row-subsampled dictionary D_s = Psi D, Psi picking the kept elements in
  increasing m1 + m2*M1 order (eqs. (6)-(7));
* the Gram D_s^H D_s, formed explicitly (eq. (17), left-hand side) or applied
  as D_s^H (D_s x) through the Kronecker factors -- steering-vector algebra,
  no FFT on the plain solvers' path;
* ISTA (eq. (9)), FISTA (eqs. (10)-(12)), ADMM (eqs. (13)-(15));
* the eigenvalues of a BCCB from its first column (eq. (21)) and the FFT
  matvec of eq. (23), used only where the paper's own "fast" formulation is
  the object of a check (Table I style comparisons).

Readings of the paper taken here (each is listed in the design notes):
  R1  objective is 1/2 ||y - D_s c||^2 + tau ||c||_1, the function whose
      proximal-gradient step is eq. (9) with mu = 1/sigma_max^2, kappa1 = mu*tau;
  R3  S_kappa(z) = 0 for |z| <= kappa;
  R4  ADMM threshold kappa2 = tau/rho (scaled ADMM; equals the printed rho*tau
      at rho = 1);
  R5  FISTA starts from alpha_1 = 1 so the first momentum weight is 0;
  R6  ADMM returns the sparse iterate z^T (and c^T);
  R9  the coefficient index is l1 + l2*L1;
  R10 DFT is unnormalised e^{-j 2 pi k n / N}, its inverse carries 1/N.

Grids are stored as numpy arrays of shape [L2][L1] (l1 fastest), i.e.
grid[l2, l1] = c[l1 + l2*L1].
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


# ---------------------------------------------------------------------------
# Grids and dictionaries (Sec. II-A, Sec. III-A)
# ---------------------------------------------------------------------------

def harmonic_grid(L: int) -> np.ndarray:
    """Uniform harmonic grid f_l = -1/2 + l/L, l = 0..L-1 (eq. (16), gamma = 1/2)."""
    return -0.5 + np.arange(L) / L


def subdictionary(M: int, L: int) -> np.ndarray:
    """D_i(m, l) = exp(-j 2 pi f_l m) for m < M, l < L (eq. (5)), complex128 [M][L].

    f_l * m = ((l - L/2) * m) / L exactly for even L, so the phase is taken from
    the integer residue ((l - L/2) * m) mod L (no drift of a float product).
    For odd L the float phase is used directly.
    """
    m = np.arange(M, dtype=np.int64)[:, None]
    l = np.arange(L, dtype=np.int64)[None, :]
    if L % 2 == 0:
        k = ((l - L // 2) * m) % L
        return np.exp(-1j * TWO_PI * k / L)
    f = harmonic_grid(L)[None, :]
    return np.exp(-1j * TWO_PI * f * m)


def sensors(mask: np.ndarray) -> np.ndarray:
    """(m1, m2) of the kept elements, increasing m1 + m2*M1 (rows of Psi, eq. (6))."""
    m2, m1 = np.nonzero(np.asarray(mask))
    return np.stack([m1, m2], axis=1).astype(np.int64)


def sparse_dictionary(mask: np.ndarray, L1: int, L2: int) -> np.ndarray:
    """D_s = Psi (D_2 kron D_1), complex128 [M][L1*L2] (eqs. (4), (7)).

    Row m (sensor (m1, m2)) of D_2 kron D_1 is D_2[m2, :] kron D_1[m1, :]; its
    entry for column l1 + l2*L1 is D_1[m1, l1] * D_2[m2, l2].
    """
    M2, M1 = mask.shape
    D1 = subdictionary(M1, L1)
    D2 = subdictionary(M2, L2)
    s = sensors(mask)
    rows = D2[s[:, 1], :][:, :, None] * D1[s[:, 0], :][:, None, :]  # [M][L2][L1]
    return rows.reshape(len(s), L1 * L2)


class Operator:
    """D_s and D_s^H applied through the Kronecker factors of eq. (4).

    D c  for c = vec(C), C[l2, l1]:  (D_2 C D_1^T)[m2, m1]   (full URA response)
    D_s c = that response at the kept elements (Psi, eq. (6)).
    D_s^H r = D_2^H R conj(D_1) with R the kept-element values placed on the
              M2 x M1 grid (zeros elsewhere).
    Cost O(M2*L1*L2 + M1*M2*L1) per product, no FFT.
    """

    def __init__(self, mask: np.ndarray, L1: int, L2: int):
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.M2, self.M1 = self.mask.shape
        self.L1, self.L2 = int(L1), int(L2)
        self.L = self.L1 * self.L2
        self.D1 = subdictionary(self.M1, self.L1)
        self.D2 = subdictionary(self.M2, self.L2)
        self.s = sensors(self.mask)
        self.M = len(self.s)

    # D_s c
    def forward(self, c: np.ndarray) -> np.ndarray:
        C = np.asarray(c, dtype=np.complex128).reshape(self.L2, self.L1)
        full = self.D2 @ C @ self.D1.T          # [M2][M1]
        return full[self.s[:, 1], self.s[:, 0]]

    # D_s^H y
    def adjoint(self, y: np.ndarray) -> np.ndarray:
        R = np.zeros((self.M2, self.M1), dtype=np.complex128)
        R[self.s[:, 1], self.s[:, 0]] = np.asarray(y, dtype=np.complex128)
        return (self.D2.conj().T @ R @ self.D1.conj()).reshape(self.L)

    # G x = D_s^H D_s x
    def gram(self, x: np.ndarray) -> np.ndarray:
        return self.adjoint(self.forward(x))

    def gram_at(self, x: np.ndarray, idx: np.ndarray) -> np.ndarray:
        """(G x)[idx] only: D_s x once, then one row of D_s^H per requested index."""
        r = self.forward(x)
        idx = np.asarray(idx, dtype=np.int64)
        l1 = idx % self.L1
        l2 = idx // self.L1
        cols = (self.D1[self.s[:, 0]][:, l1] * self.D2[self.s[:, 1]][:, l2])  # [M][n]
        return cols.conj().T @ r

    # D_s D_s^H  (M x M), separable: (D1 D1^H)[m1, m1'] (D2 D2^H)[m2, m2']
    def outer_gram(self) -> np.ndarray:
        A1 = self.D1 @ self.D1.conj().T
        A2 = self.D2 @ self.D2.conj().T
        m1 = self.s[:, 0]
        m2 = self.s[:, 1]
        return A1[np.ix_(m1, m1)] * A2[np.ix_(m2, m2)]


def gram_dense(mask: np.ndarray, L1: int, L2: int) -> np.ndarray:
    """Explicit G = D_s^H D_s, complex128 [L][L] (left-hand side of eq. (17))."""
    Ds = sparse_dictionary(mask, L1, L2)
    return Ds.conj().T @ Ds


def gram_kronecker_sum(mask: np.ndarray, L1: int, L2: int) -> np.ndarray:
    """G as the masked sum over elements of (d2 d2^H) kron (d1 d1^H) (eq. (17), last line).

    Here d_{i,m} is row m of D_i viewed as a column vector of conjugates, so that
    the sum reproduces (Psi D)^H (Psi D); used to pin gram_dense.
    """
    M2, M1 = mask.shape
    D1 = subdictionary(M1, L1)
    D2 = subdictionary(M2, L2)
    G = np.zeros((L1 * L2, L1 * L2), dtype=np.complex128)
    for m2 in range(M2):
        for m1 in range(M1):
            if mask[m2, m1]:
                a1 = D1[m1].conj()[:, None] * D1[m1][None, :]
                a2 = D2[m2].conj()[:, None] * D2[m2][None, :]
                G += np.kron(a2, a1)
    return G


# ---------------------------------------------------------------------------
# BCCB algebra (Sec. III-A, III-B)
# ---------------------------------------------------------------------------

def bccb_from_first_column(r: np.ndarray, L1: int, L2: int) -> np.ndarray:
    """The BCCB matrix with L2 x L2 blocks of L1 x L1 whose first column is r
    (property (iv)): R[(l1 + l2 L1), (l1' + l2' L1)] = r[((l1-l1') mod L1) + ((l2-l2') mod L2) L1]."""
    l1 = np.arange(L1)
    l2 = np.arange(L2)
    d1 = (l1[:, None] - l1[None, :]) % L1           # [L1][L1]
    d2 = (l2[:, None] - l2[None, :]) % L2           # [L2][L2]
    idx = d1[None, :, None, :] + L1 * d2[:, None, :, None]   # [l2][l1][l2'][l1']
    return np.asarray(r)[idx].reshape(L1 * L2, L1 * L2)


def first_column_grid(G: np.ndarray, L1: int, L2: int) -> np.ndarray:
    """R0[l2, l1] = G[l1 + l2 L1, 0]: the blocks r_{l2} of property (iv) as rows."""
    return np.asarray(G)[:, 0].reshape(L2, L1)


def eigenvalues_from_first_column(R0: np.ndarray) -> np.ndarray:
    """Omega from eq. (21): lambda_{l2'} = F_L1( sum_l2 r_l2 exp(-j 2 pi l2 l2'/L2) ).

    R0 is [L2][L1] with R0[l2] = r_{l2}.  Returns Omega as [L2][L1] with
    Omega[l2', :] = lambda_{l2'} (the paper's Omega = [lambda_0 ... lambda_{L2-1}]
    stored transposed to match the grid layout).
    """
    L2, L1 = R0.shape
    k = np.arange(L2)
    W2 = np.exp(-1j * TWO_PI * np.outer(k, k) / L2)     # L2-point DFT of the block sequence
    inner = W2 @ R0                                      # [l2'][l1]
    return np.fft.fft(inner, axis=1)                     # F_L1 of each lambda_{l2'}


def gram_first_column(op: Operator) -> np.ndarray:
    """First column r = G e_0 of the Gram, as the [L2][L1] grid R0 (no FFT)."""
    e0 = np.zeros(op.L, dtype=np.complex128)
    e0[0] = 1.0
    return op.gram(e0).reshape(op.L2, op.L1)


def bccb_eigenvalues(mask: np.ndarray, L1: int, L2: int) -> np.ndarray:
    """Gram eigenvalue grid Omega [L2][L1] (eq. (21) applied to G's first column)."""
    return eigenvalues_from_first_column(gram_first_column(Operator(mask, L1, L2)))


def fft_matvec(Omega: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The paper's fast product R c = vec(F^-1_L1 (Omega . F_L1 C F_L2^T)(F^-1_L2)^T) (eq. (23)).

    Used only to reproduce the "fast" side of the regular-vs-fast comparison
    (Table I); the plain solvers below never call it.
    """
    L2, L1 = Omega.shape
    C = np.asarray(x, dtype=np.complex128).reshape(L2, L1)
    return np.fft.ifft2(Omega * np.fft.fft2(C)).reshape(L1 * L2)


def fft_matvec_columns(Omega: np.ndarray, X: np.ndarray) -> np.ndarray:
    """eq. (23) applied to each column of X ([L][n]): column j is fft_matvec(Omega, X[:, j])."""
    L2, L1 = Omega.shape
    C = np.asarray(X, dtype=np.complex128).reshape(L2, L1, -1)
    return np.fft.ifft2(Omega[:, :, None] * np.fft.fft2(C, axes=(0, 1)), axes=(0, 1)).reshape(L1 * L2, -1)


def shifted_inverse_dense(op: "Operator", rho: float) -> np.ndarray:
    """The explicit L x L matrix (G + rho I)^-1 of eq. (13), formed by the Woodbury identity
    (1/rho)(I - D_s^H (rho I_M + D_s D_s^H)^-1 D_s) from the explicit D_s."""
    Ds = sparse_dictionary(op.mask, op.L1, op.L2)
    K = rho * np.eye(op.M) + Ds @ Ds.conj().T
    return (np.eye(op.L) - Ds.conj().T @ np.linalg.solve(K, Ds)) / rho


def dft_matrix(N: int) -> np.ndarray:
    k = np.arange(N)
    return np.exp(-1j * TWO_PI * np.outer(k, k) / N)


def bccb_diagonalisation(Omega: np.ndarray) -> np.ndarray:
    """R = (F_L2^-1 kron I_L1) Gamma^-1 Lambda Gamma (F_L2 kron I_L1) (eqs. (18)-(20)),
    with Gamma = diag(F_L1, ..., F_L1) and Lambda = diag(diag(lambda_0), ...)."""
    L2, L1 = Omega.shape
    F1 = dft_matrix(L1)
    F2 = dft_matrix(L2)
    I1 = np.eye(L1)
    Gam = np.kron(np.eye(L2), F1)
    Gam_inv = np.kron(np.eye(L2), np.linalg.inv(F1))
    Lam = np.diag(Omega.reshape(-1))
    A = np.kron(F2, I1)
    A_inv = np.kron(np.linalg.inv(F2), I1)
    return A_inv @ Gam_inv @ Lam @ Gam @ A


# ---------------------------------------------------------------------------
# LASSO pieces (Sec. II-B)
# ---------------------------------------------------------------------------

def step_size(op: Operator) -> float:
    """mu = 1 / sigma_max(D_s)^2, sigma_max^2 = largest eigenvalue of D_s D_s^H (eq. (9))."""
    return 1.0 / float(np.linalg.eigvalsh(op.outer_gram())[-1])


def soft_threshold(z: np.ndarray, kappa) -> np.ndarray:
    """S_kappa(z) = exp(j arg z) max(|z| - kappa, 0), and 0 where |z| <= kappa (R3).

    kappa may be an array broadcasting against z (e.g. one threshold per column when the
    columns of z are independent problems); each element is thresholded by its own kappa."""
    z = np.asarray(z, dtype=np.complex128)
    a = np.abs(z)
    out = np.zeros_like(z)
    keep = a > kappa
    k = np.broadcast_to(kappa, z.shape)[keep] if np.ndim(kappa) else kappa
    out[keep] = z[keep] * (1.0 - k / a[keep])
    return out


def objective(op: Operator, y: np.ndarray, c: np.ndarray, tau: float) -> float:
    """F(c) = 1/2 ||y_s - D_s c||^2 + tau ||c||_1 (eq. (8) under reading R1)."""
    r = np.asarray(y, dtype=np.complex128) - op.forward(c)
    return 0.5 * float(np.vdot(r, r).real) + tau * float(np.abs(c).sum())


def kkt_residual(op: Operator, b: np.ndarray, c: np.ndarray, tau: float, Gc=None):
    """LASSO stationarity residual of c.

    g = b - G c.  e_l = |g_l - tau c_l/|c_l|| if c_l != 0, else max(|g_l| - tau, 0).
    Returns (||e||_2 / ||b||_2, max_l e_l / tau).  Both are 0 exactly at a minimiser.
    """
    c = np.asarray(c, dtype=np.complex128)
    g = np.asarray(b) - (op.gram(c) if Gc is None else Gc)
    a = np.abs(c)
    nz = a > 0
    e = np.empty(c.shape, dtype=np.float64)
    e[nz] = np.abs(g[nz] - tau * c[nz] / a[nz])
    e[~nz] = np.maximum(np.abs(g[~nz]) - tau, 0.0)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(e)) / nb, (float(e.max()) / tau if tau > 0 else float(e.max()))


def fista_weights(iters: int) -> np.ndarray:
    """Momentum weights beta_t = (alpha_t - 1)/alpha_{t+1}, t = 1..iters, from
    alpha_1 = 1 and alpha_{t+1} = (1 + sqrt(1 + 4 alpha_t^2))/2 (eqs. (11)-(12), R5)."""
    beta = np.empty(iters, dtype=np.float64)
    a = 1.0
    for t in range(iters):
        a_next = (1.0 + np.sqrt(1.0 + 4.0 * a * a)) / 2.0
        beta[t] = (a - 1.0) / a_next
        a = a_next
    return beta


def ista(apply_G, b, mu: float, tau: float, iters: int, c0=None, trace=None):
    """ISTA, eq. (9): c <- S_{mu tau}(c - mu G c + mu b); returns c^(iters)."""
    c = np.zeros_like(b) if c0 is None else np.array(c0, dtype=np.complex128)
    kappa = mu * tau
    for _ in range(iters):
        c = soft_threshold(c - mu * apply_G(c) + mu * b, kappa)
        if trace is not None:
            trace(c)
    return c


def fista(apply_G, b, mu: float, tau: float, iters: int, c0=None, trace=None):
    """FISTA, eqs. (10)-(12): z^1 = c^0; c^t = S_{mu tau}(z^t - mu G z^t + mu b);
    z^{t+1} = c^t + beta_t (c^t - c^{t-1}).  Exactly `iters` Gram products."""
    c_prev = np.zeros_like(b) if c0 is None else np.array(c0, dtype=np.complex128)
    z = c_prev.copy()
    kappa = mu * tau
    beta = fista_weights(iters)
    c = c_prev
    for t in range(iters):
        c = soft_threshold(z - mu * apply_G(z) + mu * b, kappa)
        z = c + beta[t] * (c - c_prev)
        c_prev = c
        if trace is not None:
            trace(c)
    return c


class ShiftedInverse:
    """x -> (G + rho I)^-1 x for the ADMM c-update (eq. (13)).

    Small L: Cholesky of the explicit Hermitian positive definite G + rho I.
    Large L: Woodbury, (1/rho)(I - D_s^H (rho I_M + D_s D_s^H)^-1 D_s).
    """

    def __init__(self, op: Operator, rho: float, dense_limit: int = 4096):
        self.op = op
        self.rho = float(rho)
        self.dense = op.L <= dense_limit
        if self.dense:
            G = gram_dense(op.mask, op.L1, op.L2)
            self.chol = np.linalg.cholesky(G + rho * np.eye(op.L))
        else:
            self.small = np.linalg.inv(rho * np.eye(op.M) + op.outer_gram())

    def __call__(self, x):
        x = np.asarray(x, dtype=np.complex128)
        if self.dense:
            t = np.linalg.solve(self.chol, x)
            return np.linalg.solve(self.chol.conj().T, t)
        return (x - self.op.adjoint(self.small @ self.op.forward(x))) / self.rho


def admm(apply_inv, b, rho: float, tau: float, iters: int, trace=None):
    """ADMM, eqs. (13)-(15) with kappa2 = tau/rho (R4), z^0 = v^0 = 0.

    c^{t+1} = (G + rho I)^-1 (b + rho (z^t - v^t)), with (G + rho I)^-1 b
    precomputed once; z^{t+1} = S_{tau/rho}(c^{t+1} + v^t); v^{t+1} = v^t + c^{t+1} - z^{t+1}.
    Returns (z^T, c^T)."""
    w = apply_inv(b)
    z = np.zeros_like(b)
    v = np.zeros_like(b)
    c = np.zeros_like(b)
    kappa = tau / rho
    for _ in range(iters):
        c = w + rho * apply_inv(z - v)
        z = soft_threshold(c + v, kappa)
        v = v + c - z
        if trace is not None:
            trace(z, c, v)
    return z, c


def converged_reference(op: Operator, b, mu, tau, tol=1e-8, max_iters=200000, check=50):
    """FISTA run until max e/tau <= tol (or max_iters): the converged LASSO c*."""
    apply_G = op.gram
    c_prev = np.zeros_like(b)
    z = c_prev.copy()
    a = 1.0
    kappa = mu * tau
    for t in range(max_iters):
        c = soft_threshold(z - mu * apply_G(z) + mu * b, kappa)
        a_next = (1.0 + np.sqrt(1.0 + 4.0 * a * a)) / 2.0
        z = c + ((a - 1.0) / a_next) * (c - c_prev)
        a = a_next
        c_prev = c
        if (t + 1) % check == 0:
            _, mx = kkt_residual(op, b, c, tau)
            if mx <= tol:
                return c, t + 1
    return c_prev, max_iters


# ---------------------------------------------------------------------------
# Convenience: a whole problem instance
# ---------------------------------------------------------------------------

class Problem:
    """One scene's LASSO in FP64: D_s, b = D_s^H y_s, mu, tau."""

    def __init__(self, mask, L1, L2, y, tau=None, tau_fraction=0.1, dense=None):
        self.op = Operator(mask, L1, L2)
        self.y = np.asarray(y, dtype=np.complex64).astype(np.complex128)
        self.b = self.op.adjoint(self.y)
        self.mu = step_size(self.op)
        if tau is None:
            tau = np.float32(tau_fraction * np.abs(self.b).max())
        self.tau = float(np.float32(tau))
        if dense is None:
            dense = self.op.L <= 4096
        self.G = gram_dense(mask, L1, L2) if dense else None

    def apply_G(self, x):
        return self.G @ x if self.G is not None else self.op.gram(x)

    def ista(self, iters, c0=None):
        return ista(self.apply_G, self.b, self.mu, self.tau, iters, c0)

    def fista(self, iters, c0=None):
        return fista(self.apply_G, self.b, self.mu, self.tau, iters, c0)

    def admm(self, rho, iters):
        return admm(ShiftedInverse(self.op, rho), self.b, rho, self.tau, iters)

    def objective(self, c):
        return objective(self.op, self.y, c, self.tau)

    def kkt(self, c):
        return kkt_residual(self.op, self.b, c, self.tau)
