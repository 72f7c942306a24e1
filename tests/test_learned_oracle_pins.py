"""Pins of the learned-FISTA oracle: reduction to plain FISTA, the filter convolution
against a dense spatial-domain construction, and the hand-derived backward against
central finite differences."""
import numpy as np

from oracle import bccb_oracle as O
from oracle import learned_oracle as LO
from paper_2509_13592_amd import scenes as S


def _problem(seed=0, L=16, M1=5, M2=4, kept=10):
    sc = S.custom_scene(M1, M2, kept, L, L, K=2, snr_db=20, seed=(21, seed, L))
    P = O.Problem(sc.mask, L, L, sc.y)
    Om = O.bccb_eigenvalues(sc.mask, L, L)
    return sc, P, Om


def test_identity_params_reduce_to_fista():
    """s = theta = 1, Delta = 0: every layer is one FISTA iteration of eqs. (10)-(12)."""
    sc, P, Om = _problem(L=32, M1=8, M2=8, kept=32)
    K = 7
    c = LO.forward(Om, P.mu, LO.init_params(K), P.b.reshape(32, 32), P.tau)
    ref = P.fista(K)
    assert np.abs(c.reshape(-1) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_layer_filter_against_dense_bccb():
    """A layer with a random 5x5 Delta equals u = (I - mu G') z + mu b where G' is the dense
    BCCB whose first column is the Gram's first column r modulated by the taps:
    r'(l) = r(l) (1 + sum_ab Delta[a,b] e^{+j2pi(a l2/L2 + b l1/L1)}) (a spectral shift by
    (a, b) is a modulation of the first column)."""
    sc, P, Om = _problem(seed=1, L=16)
    L1 = L2 = 16
    rng = np.random.default_rng(3)
    p = LO.init_params(1)
    p[0, 0] = 0.8
    p[0, 2:] = 0.05 * rng.standard_normal(50)
    _, _, d = LO.unpack(p[0])
    G = O.gram_dense(sc.mask, L1, L2)
    r = G[:, 0].reshape(L2, L1)
    l2, l1 = np.meshgrid(np.arange(L2), np.arange(L1), indexing="ij")
    mod = np.ones((L2, L1), dtype=complex)
    for a in range(-2, 3):
        for b in range(-2, 3):
            mod += d[a + 2, b + 2] * np.exp(2j * np.pi * (a * l2 / L2 + b * l1 / L1))
    Gp = O.bccb_from_first_column((r * mod).reshape(-1), L1, L2)
    mu = 0.8 * P.mu
    z = (rng.standard_normal(L1 * L2) + 1j * rng.standard_normal(L1 * L2))
    want = z - mu * (Gp @ z) + mu * P.b
    mu_o, th, Om_p, m = LO.layer_spectrum(Om, P.mu, p[0])
    got = np.fft.ifft2(m * np.fft.fft2(z.reshape(L2, L1))) + mu_o * P.b.reshape(L2, L1)
    assert np.abs(got.reshape(-1) - want).max() <= 1e-10 * np.abs(want).max()


def test_backward_matches_finite_differences():
    K = 3
    L = 16
    scs = [_problem(seed=s, L=L) for s in (4, 5)]
    Om = scs[0][2]
    mu0 = scs[0][1].mu
    # both scenes share the first scene's mask (one geometry), own snapshots
    mask = scs[0][0].mask
    bs, taus, labels = [], [], []
    rng = np.random.default_rng(7)
    for s in (4, 5):
        sc = S.custom_scene(5, 4, 10, L, L, K=2, snr_db=20, seed=(22, s, L), mask=mask)
        P = O.Problem(mask, L, L, sc.y)
        bs.append(P.b.reshape(L, L))
        taus.append(P.tau)
        labels.append(P.fista(40).reshape(L, L))
    params = LO.init_params(K)
    params[:, 0] += 0.1 * rng.standard_normal(K)
    params[:, 1] += 0.1 * rng.standard_normal(K)
    params[:, 2:] = 0.03 * rng.standard_normal((K, 50))
    loss, g = LO.loss_and_grad(Om, mu0, params, bs, taus, labels)
    h = 1e-6
    fd = np.zeros_like(params)
    for k in range(K):
        for j in range(params.shape[1]):
            pp = params.copy()
            pm = params.copy()
            pp[k, j] += h
            pm[k, j] -= h
            lp, _ = LO.loss_and_grad(Om, mu0, pp, bs, taus, labels)
            lm, _ = LO.loss_and_grad(Om, mu0, pm, bs, taus, labels)
            fd[k, j] = (lp - lm) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    assert np.abs(g - fd).max() <= 1e-5 * scale, np.abs(g - fd).max() / scale
