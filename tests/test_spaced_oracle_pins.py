"""Pins of the spaced-grid oracle (general element spacing gamma, any grid length).

The checks come from outside the oracle: the grid definition of eq. (16) evaluated as
plain floats, the steering model of eq. (2), closed forms of the geometric sums the Gram
entries are (full URA), the block-Toeplitz structure by brute force, an SVD of the
explicit D_s for the step, the matched-filter peak of an on-grid target, and the LASSO
optimality conditions.  At gamma = 1/2 the spaced oracle must reproduce the BCCB oracle.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import bccb_oracle as O
from oracle import spaced_oracle as SO
from paper_2509_13592_amd import scenes as S

GAMMAS = [Fraction(1, 4), Fraction(3, 8), Fraction(2, 5)]


def _mask(M1, M2, M, seed=0):
    return S.custom_scene(M1, M2, M, 8, 8, K=1, snr_db=20, seed=(97, seed, M1 * 100 + M2)).mask


def _crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("L", [8, 32, 12, 7])
def test_half_spacing_reproduces_bccb_dictionary(L):
    """gamma = 1/2 is the grid of the BCCB oracle: identical for even L, to rounding for odd L."""
    D = SO.subdictionary(9, L, Fraction(1, 2))
    ref = O.subdictionary(9, L)
    if L % 2 == 0:
        assert np.array_equal(D, ref)
    else:
        assert np.abs(D - ref).max() <= 1e-13


@pytest.mark.parametrize("gamma", GAMMAS)
@pytest.mark.parametrize("L", [16, 12])
def test_dictionary_is_the_steering_vector_on_the_grid(gamma, L):
    """Column l of D_i is a_i(f_l) of eq. (3) with f_l = -gamma + l 2 gamma / L (eq. (16)),
    evaluated here with plain float harmonics; the grid spans [-gamma, gamma)."""
    M = 11
    f = -float(gamma) + np.arange(L) * 2.0 * float(gamma) / L
    assert np.allclose(SO.harmonic_grid(L, gamma), f, rtol=0, atol=1e-15)
    assert f[0] == -float(gamma) and f[-1] < float(gamma)
    a = np.exp(-2j * np.pi * np.outer(np.arange(M), f))
    assert np.abs(SO.subdictionary(M, L, gamma) - a).max() <= 1e-12


@pytest.mark.parametrize("gamma1,gamma2", [(Fraction(1, 4), Fraction(3, 8)), (Fraction(2, 5), Fraction(1, 2))])
def test_gram_is_block_toeplitz_not_circulant(gamma1, gamma2):
    """G = D_s^H D_s depends only on (l1 - l1', l2 - l2') (block Toeplitz, Toeplitz blocks) on
    the uniform grid (Sec. III-A); with a spacing below 1/2 it is not circulant."""
    mask = _mask(5, 4, 13)
    L1, L2 = 12, 8
    op = SO.Operator(mask, L1, L2, gamma1, gamma2)
    G = SO.gram_dense(op).reshape(L2, L1, L2, L1)
    for d2 in range(-(L2 - 1), L2):
        for d1 in range(-(L1 - 1), L1):
            vals = [G[a2, a1, a2 - d2, a1 - d1]
                    for a2 in range(max(0, d2), min(L2, L2 + d2))
                    for a1 in range(max(0, d1), min(L1, L1 + d1))]
            assert np.abs(np.array(vals) - vals[0]).max() <= 1e-12 * op.M
    # circulant would need G[l, l'] to depend on the differences mod L; it does not
    circ = O.bccb_from_first_column(G.reshape(L1 * L2, L1 * L2)[:, 0], L1, L2)
    assert np.abs(circ - G.reshape(L1 * L2, L1 * L2)).max() > 0.1


@pytest.mark.parametrize("gamma", GAMMAS + [Fraction(1, 2)])
def test_full_ura_gram_closed_form(gamma):
    """Full URA: G = (D_2^H D_2) kron (D_1^H D_1) with (D_i^H D_i)[l, l'] the geometric sum
    sum_{m<M} e^{j theta m}, theta = 2 pi 2 gamma (l - l') / L, i.e. M or
    (1 - e^{j theta M}) / (1 - e^{j theta})."""
    M1, M2, L1, L2 = 6, 4, 10, 8
    mask = np.ones((M2, M1), dtype=np.uint8)
    op = SO.Operator(mask, L1, L2, gamma, gamma)

    def toe(M, L):
        d = np.arange(L)[:, None] - np.arange(L)[None, :]
        th = 2 * np.pi * 2 * float(gamma) * d / L
        with np.errstate(invalid="ignore", divide="ignore"):
            v = (1 - np.exp(1j * th * M)) / (1 - np.exp(1j * th))
        return np.where(np.abs(np.exp(1j * th) - 1) < 1e-12, M, v)

    want = np.kron(toe(M2, L2), toe(M1, L1))
    assert np.abs(SO.gram_dense(op) - want).max() <= 1e-11


@pytest.mark.parametrize("gamma1,gamma2", [(Fraction(1, 4), Fraction(1, 4)), (Fraction(3, 8), Fraction(2, 5))])
def test_step_from_svd(gamma1, gamma2):
    """mu = 1/sigma_max(D_s)^2: the oracle's eigvalsh of D_s D_s^H against an SVD of D_s."""
    op = SO.Operator(_mask(6, 5, 17), 12, 10, gamma1, gamma2)
    smax = np.linalg.svd(SO.sparse_dictionary(op), compute_uv=False)[0]
    assert abs(O.step_size(op) * smax ** 2 - 1.0) <= 1e-12


@pytest.mark.parametrize("gamma", GAMMAS)
def test_matched_filter_peak_of_on_grid_target(gamma):
    """A noiseless target exactly on grid point (l1*, l2*) gives b = D_s^H y peaking at that
    index with value M c (every kept element adds |a|^2 = 1): pins the sign and the index
    order of f against the steering model of eq. (2)."""
    mask = _mask(7, 6, 25)
    L1, L2 = 16, 12
    op = SO.Operator(mask, L1, L2, gamma, gamma)
    l1s, l2s = 5, 9
    f1 = -float(gamma) + l1s * 2 * float(gamma) / L1
    f2 = -float(gamma) + l2s * 2 * float(gamma) / L2
    s = O.sensors(mask)
    c = 0.7 - 0.2j
    y = c * np.exp(-2j * np.pi * (s[:, 0] * f1 + s[:, 1] * f2))
    b = op.adjoint(y)
    assert int(np.argmax(np.abs(b))) == l1s + l2s * L1
    assert abs(b[l1s + l2s * L1] - op.M * c) <= 1e-12 * op.M


def test_spaced_lasso_minimiser_and_solvers_agree():
    """At gamma = (1/4, 3/8): ISTA and FISTA approach one minimiser (objective values agree,
    the KKT residual of the FISTA iterate is small), and ADMM reaches it too."""
    sc = S.spaced_scene(0.25, 0.375, 6, 5, 17, 12, 10, K=3, snr_db=20.0)
    P = SO.Problem(sc.mask, sc.L1, sc.L2, sc.y, Fraction(1, 4), Fraction(3, 8))
    cf = P.fista(3000)
    ci = P.ista(20000)
    za, _ = P.admm(4.0, 4000)
    Ff = P.objective(cf)
    assert abs(P.objective(ci) - Ff) <= 1e-7 * Ff
    assert abs(P.objective(za) - Ff) <= 1e-7 * Ff
    r, mx = P.kkt(cf)
    assert mx <= 1e-5, (r, mx)


def test_spaced_ista_objective_monotone():
    sc = S.spaced_scene(0.25, 0.25, 5, 5, 14, 10, 12, K=2, snr_db=15.0, seed=(7, 0, 1))
    P = SO.Problem(sc.mask, sc.L1, sc.L2, sc.y, Fraction(1, 4), Fraction(1, 4))
    F = []
    c = np.zeros(P.op.L, dtype=complex)
    for _ in range(60):
        c = O.ista(P.apply_G, P.b, P.mu, P.tau, 1, c0=c)
        F.append(P.objective(c))
    assert all(F[i + 1] <= F[i] * (1 + 1e-12) for i in range(len(F) - 1))


@pytest.mark.parametrize("M1,M2,M,L1,L2", [(5, 3, 9, 12, 6), (4, 4, 11, 10, 7), (7, 3, 12, 6, 5)])
def test_non_power_of_two_grid_is_bccb_with_fold_eigenvalues(M1, M2, M, L1, L2):
    """gamma = 1/2 on grid lengths that are not powers of two (some odd): G is still the BCCB
    of its first column (eq. (17)) and eq. (21)'s eigenvalues are L1 L2 x the fold count."""
    mask = _mask(M1, M2, M)
    op = SO.Operator(mask, L1, L2)
    G = SO.gram_dense(op)
    assert np.abs(G - O.bccb_from_first_column(G[:, 0], L1, L2)).max() <= 1e-12 * op.M
    fold = np.zeros((L2, L1))
    for m1, m2 in O.sensors(mask):
        fold[m2 % L2, m1 % L1] += 1
    Om = O.eigenvalues_from_first_column(G[:, 0].reshape(L2, L1))
    assert np.abs(Om - L1 * L2 * fold).max() <= 1e-9 * L1 * L2
    x = _crandn(np.random.default_rng(4), op.L)
    assert np.linalg.norm(op.gram(x) - G @ x) <= 1e-12 * np.linalg.norm(G @ x)
