"""FP64 reference of the learned unrolled FISTA and its hand-derived backward.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Network (the learned extension of FISTA, eqs. (10)-(12); each layer keeps the
BCCB structure because BCCBs are closed under linear combination, Sec. III-A (i)):

  z_0 = 0, c_{-1} = 0, for layer k = 0 .. K-1:
    Omega'_k = Omega + Delta_k (*) Omega           (5x5 complex circular conv, centred)
    m_k      = 1 - mu_k Omega'_k                    (complex spectrum of layer k)
    u_k      = IDFT2(m_k . DFT2(z_k)) + mu_k b      (b = D_s^H y)
    c_k      = S_{kappa_k}(u_k),  kappa_k = theta_k mu_k tau
    z_{k+1}  = c_k + beta_k (c_k - c_{k-1})         (beta_k: the FISTA schedule, beta_0 = 0)
  output c_{K-1}.

Parameters per layer: s_k (mu_k = s_k mu0, mu0 = 1/max Omega), theta_k, Delta_k in
C^{5x5}.  With s = theta = 1 and Delta = 0 every layer is exactly one FISTA
iteration (pinned against the steering-vector FISTA of bccb_oracle).

Loss: mean over scenes of ||c_{K-1} - c*||^2 / ||c*||^2.

Gradient convention for a real loss of complex x: g = dl/dRe(x) + j dl/dIm(x),
so that dl = Re(sum conj(g) dx).  The trained weights are not a pinned
quantity: only the forward/backward arithmetic is pinned (finite differences).
"""
from __future__ import annotations

import numpy as np

from .bccb_oracle import fista_weights, soft_threshold

TAPS = 5
HALF = TAPS // 2
PER_LAYER = 2 + 2 * TAPS * TAPS      # s, theta, Re/Im Delta[5][5]


def init_params(layers: int) -> np.ndarray:
    p = np.zeros((layers, PER_LAYER), dtype=np.float64)
    p[:, 0] = 1.0
    p[:, 1] = 1.0
    return p


def unpack(p_layer):
    s, th = float(p_layer[0]), float(p_layer[1])
    d = np.asarray(p_layer[2:2 + TAPS * TAPS]) + 1j * np.asarray(p_layer[2 + TAPS * TAPS:])
    return s, th, d.reshape(TAPS, TAPS)


def conv_filter(Omega: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """(Delta (*) Omega)[k2, k1] = sum_{a,b=-2..2} Delta[a+2, b+2] Omega[(k2-a) mod L2, (k1-b) mod L1]."""
    out = np.zeros(Omega.shape, dtype=np.complex128)
    for a in range(-HALF, HALF + 1):
        for b in range(-HALF, HALF + 1):
            w = delta[a + HALF, b + HALF]
            if w != 0:
                out += w * np.roll(np.roll(Omega, a, axis=0), b, axis=1)
    return out


def layer_spectrum(Omega, mu0, p_layer):
    s, th, d = unpack(p_layer)
    mu = s * mu0
    Om_p = Omega + conv_filter(Omega, d)
    return mu, th, Om_p, 1.0 - mu * Om_p


def forward(Omega, mu0, params, b, tau, save=False):
    """b: [L2][L1] complex (one scene); returns c_{K-1} (and the saved activations)."""
    K = params.shape[0]
    beta = fista_weights(K)
    z = np.zeros_like(b)
    c_prev = np.zeros_like(b)
    acts = []
    c = c_prev
    for k in range(K):
        mu, th, Om_p, m = layer_spectrum(Omega, mu0, params[k])
        u = np.fft.ifft2(m * np.fft.fft2(z)) + mu * b
        kappa = th * mu * tau
        c = soft_threshold(u, kappa)
        acts.append((z, u, c, m, mu, th, kappa, Om_p))
        z = c + beta[k] * (c - c_prev)
        c_prev = c
    return (c, acts) if save else c


def shrink_vjp(u, kappa, g):
    """Vector-Jacobian product of S_kappa at u applied to g, and d/dkappa (summed)."""
    a = np.abs(u)
    keep = a > kappa
    gu = np.zeros_like(u)
    ak = a[keep]
    uk = u[keep]
    gk = g[keep]
    proj = np.real(np.conj(uk) * gk)
    gu[keep] = (1.0 - kappa / ak) * gk + kappa * proj * uk / ak ** 3
    gkappa = -float(np.sum(proj / ak))
    return gu, gkappa


def backward(Omega, mu0, params, b, tau, acts, gc_out):
    """Gradient of a real loss w.r.t. params given g = dl/dc_{K-1} (convention above)."""
    K = params.shape[0]
    L = Omega.size
    beta = fista_weights(K)
    grads = np.zeros_like(params)
    gz_next = np.zeros_like(b)     # dl/dz_{k+1}
    gz_next2 = np.zeros_like(b)    # dl/dz_{k+2}
    for k in range(K - 1, -1, -1):
        z, u, c, m, mu, th, kappa, Om_p = acts[k]
        gc = (1.0 + beta[k]) * gz_next
        if k + 1 < K:
            gc = gc - beta[k + 1] * gz_next2
        if k == K - 1:
            gc = gc + gc_out
        gu, gkappa = shrink_vjp(u, kappa, gc)
        U = np.fft.fft2(gu)
        Z = np.fft.fft2(z)
        gm = U * np.conj(Z) / L                       # dl/dm_k
        gmu = -float(np.real(np.sum(np.conj(gm) * Om_p)))
        gmu += float(np.real(np.sum(np.conj(gu) * b)))
        gmu += gkappa * th * tau
        gth = gkappa * mu * tau
        gOm = -mu * gm                                # dl/dOmega'_k
        gd = np.zeros((TAPS, TAPS), dtype=np.complex128)
        for a in range(-HALF, HALF + 1):
            for bb in range(-HALF, HALF + 1):
                sh = np.roll(np.roll(Omega, a, axis=0), bb, axis=1)
                gd[a + HALF, bb + HALF] = np.sum(gOm * np.conj(sh))
        grads[k, 0] = gmu * mu0
        grads[k, 1] = gth
        grads[k, 2:2 + TAPS * TAPS] = gd.real.reshape(-1)
        grads[k, 2 + TAPS * TAPS:] = gd.imag.reshape(-1)
        gz = np.fft.ifft2(np.conj(m) * U)             # H_k^H gu
        gz_next2 = gz_next
        gz_next = gz
    return grads


def loss_and_grad(Omega, mu0, params, bs, taus, labels):
    """Mean relative squared error over scenes and its parameter gradient."""
    n = len(bs)
    total = 0.0
    grads = np.zeros_like(params)
    for b, tau, lab in zip(bs, taus, labels):
        c, acts = forward(Omega, mu0, params, b, tau, save=True)
        nl = float(np.sum(np.abs(lab) ** 2))
        total += float(np.sum(np.abs(c - lab) ** 2)) / nl
        g = 2.0 * (c - lab) / nl / n
        grads += backward(Omega, mu0, params, b, tau, acts, g)
    return total / n, grads
