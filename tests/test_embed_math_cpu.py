"""Host FP64 arithmetic of the padded-embedding plans (csrc/embed_math.cpp, built here with
g++ on its own, no HIP) against the spaced-grid oracle.

The library's steering tables must be the oracle's subdictionaries (eq. (5) on the grid of
eq. (16)); the eigenvalues it computes in closed form for the circulant embedding of the
block-Toeplitz Gram must equal an FFT of the embedding built entry by entry from the oracle's
explicit Gram; the embedded (G + rho I)^-1 spectrum must come out of the oracle's explicit
inverse the same way; and its Lanczos step must match the oracle's eigvalsh of D_s D_s^H.
"""
import ctypes
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import bccb_oracle as O
from oracle import spaced_oracle as SO
from paper_2509_13592_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_13592_amd", "csrc")
CAPI = os.path.join(ROOT, "tests", "native", "embed_math_capi.cpp")

_d = ctypes.c_double
_i = ctypes.c_int
_vp = ctypes.c_void_p


@pytest.fixture(scope="module")
def em(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    so = str(tmp_path_factory.mktemp("em") / "libembed_math.so")
    cmd = ["g++", "-std=c++17", "-O2", "-shared", "-fPIC", f"-I{CSRC}", CAPI,
           os.path.join(CSRC, "embed_math.cpp"), "-o", so]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    lib = ctypes.CDLL(so)
    lib.em_embed_length.argtypes = [_i]
    lib.em_spacing_fraction.argtypes = [_d, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
    lib.em_dirichlet_exact.restype = _d
    lib.em_dirichlet_exact.argtypes = [ctypes.c_long, ctypes.c_long, _i]
    lib.em_steering.argtypes = [_i, _i, _d, _vp]
    lib.em_toeplitz_spectrum.argtypes = [_vp, _i, _i, _i, _i, _d, _d, _i, _i, _vp]
    lib.em_circulant_eigenvalues.argtypes = [_vp, _i, _i, _i, _i, _vp]
    lib.em_shifted_inverse_spectrum.argtypes = [_vp, _i, _i, _d, _i, _i, _vp]
    lib.em_gram_max_eigenvalue.restype = _d
    lib.em_gram_max_eigenvalue.argtypes = [_vp, _i, _i, _i, _i, _d, _d]
    return lib


def _mask(M1, M2, M, seed=0):
    return np.ascontiguousarray(
        S.custom_scene(M1, M2, M, 8, 8, K=1, snr_db=20, seed=(96, seed, M1 * 100 + M2)).mask, dtype=np.uint8)


def _embedded_first_column(G, L1, L2, P1, P2):
    """c_e[d2 mod P2][d1 mod P1] = G[(a1, a2), (b1, b2)] with a - b = d (any such pair)."""
    G4 = G.reshape(L2, L1, L2, L1)
    c = np.zeros((P2, P1), dtype=complex)
    for d2 in range(-(L2 - 1), L2):
        for d1 in range(-(L1 - 1), L1):
            a1, b1 = max(d1, 0), max(-d1, 0)
            a2, b2 = max(d2, 0), max(-d2, 0)
            c[d2 % P2, d1 % P1] = G4[a2, a1, b2, b1]
    return c


def test_embed_length_and_fractions(em):
    assert [em.em_embed_length(L) for L in (2, 4, 5, 8, 12, 33, 256, 512)] == [8, 8, 16, 16, 32, 128, 512, 1024]
    p, q = ctypes.c_long(), ctypes.c_long()
    for g, want in ((0.5, (1, 2)), (0.25, (1, 4)), (0.4, (2, 5)), (0.375, (3, 8)), (1.0 / 3.0, (1, 3))):
        assert em.em_spacing_fraction(g, ctypes.byref(p), ctypes.byref(q)) == 1
        assert (p.value, q.value) == want
    assert em.em_spacing_fraction(np.pi / 10, ctypes.byref(p), ctypes.byref(q)) == 0


@pytest.mark.parametrize("L", [3, 8, 12])
def test_dirichlet_sum(em, L):
    N = 97
    for n in (0, 1, 5, 50, 96, -3, 194):
        want = sum(np.exp(2j * np.pi * d * n / N) for d in range(-(L - 1), L)).real
        assert abs(em.em_dirichlet_exact(n, N, L) - want) <= 1e-12 * (2 * L)


@pytest.mark.parametrize("gamma", [0.25, 0.4, 0.5, np.pi / 10])
@pytest.mark.parametrize("L", [12, 16])
def test_steering_table_is_the_subdictionary(em, gamma, L):
    M = 9
    out = np.empty(2 * M * L)
    em.em_steering(M, L, gamma, out.ctypes.data)
    W = (out[0::2] + 1j * out[1::2]).reshape(M, L)
    g = Fraction(gamma).limit_denominator(1 << 20) if gamma != np.pi / 10 else gamma
    ref = SO.subdictionary(M, L, g) if not isinstance(g, float) else np.exp(
        -2j * np.pi * np.outer(np.arange(M), -gamma + np.arange(L) * 2 * gamma / L))
    assert np.abs(W - ref).max() <= 1e-12


@pytest.mark.parametrize("gamma1,gamma2,M1,M2,M,L1,L2", [
    (0.25, 0.375, 5, 4, 13, 12, 8),
    (0.4, 0.4, 6, 5, 17, 10, 7),
    (0.5, 0.5, 5, 3, 9, 12, 6),      # circulant, not a power of two
    (0.5, 0.25, 4, 4, 10, 8, 9),
])
def test_toeplitz_embedding_spectrum(em, gamma1, gamma2, M1, M2, M, L1, L2):
    mask = _mask(M1, M2, M)
    P1, P2 = em.em_embed_length(L1), em.em_embed_length(L2)
    out = np.empty(P1 * P2)
    em.em_toeplitz_spectrum(mask.ctypes.data, M1, M2, L1, L2, gamma1, gamma2, P1, P2, out.ctypes.data)
    g1 = Fraction(gamma1).limit_denominator(1 << 20)
    g2 = Fraction(gamma2).limit_denominator(1 << 20)
    op = SO.Operator(mask, L1, L2, g1, g2)
    G = SO.gram_dense(op)
    want = np.fft.fft2(_embedded_first_column(G, L1, L2, P1, P2))
    assert np.abs(want.imag).max() <= 1e-9 * op.M
    assert np.abs(out.reshape(P2, P1) - want.real).max() <= 1e-9 * op.M * L1 * L2 / 10


@pytest.mark.parametrize("M1,M2,M,L1,L2,rho", [(5, 3, 9, 12, 6, 1.0), (4, 4, 11, 10, 7, 0.5), (3, 3, 7, 6, 5, 40.0)])
def test_shifted_inverse_embedding_spectrum(em, M1, M2, M, L1, L2, rho):
    mask = _mask(M1, M2, M)
    P1, P2 = em.em_embed_length(L1), em.em_embed_length(L2)
    om = np.empty(L1 * L2)
    em.em_circulant_eigenvalues(mask.ctypes.data, M1, M2, L1, L2, om.ctypes.data)
    op = SO.Operator(mask, L1, L2)
    G = SO.gram_dense(op)
    assert np.abs(om.reshape(L2, L1) - O.eigenvalues_from_first_column(G[:, 0].reshape(L2, L1)).real).max() \
        <= 1e-9 * L1 * L2
    out = np.empty(P1 * P2)
    em.em_shifted_inverse_spectrum(om.ctypes.data, L1, L2, rho, P1, P2, out.ctypes.data)
    Minv = np.linalg.inv(G + rho * np.eye(op.L))
    want = np.fft.fft2(_embedded_first_column(Minv, L1, L2, P1, P2))
    assert np.abs(out.reshape(P2, P1) - want.real).max() <= 1e-11 / rho * 10


@pytest.mark.parametrize("gamma1,gamma2,M1,M2,M,L1,L2", [
    (0.25, 0.375, 6, 5, 17, 12, 10), (0.4, 0.25, 8, 8, 40, 16, 16), (0.3, 0.45, 7, 4, 20, 9, 11)])
def test_lanczos_step_matches_eigvalsh(em, gamma1, gamma2, M1, M2, M, L1, L2):
    mask = _mask(M1, M2, M)
    lam = em.em_gram_max_eigenvalue(mask.ctypes.data, M1, M2, L1, L2, gamma1, gamma2)
    op = SO.Operator(mask, L1, L2, Fraction(gamma1).limit_denominator(1 << 20),
                     Fraction(gamma2).limit_denominator(1 << 20))
    assert abs(lam * O.step_size(op) - 1.0) <= 1e-11
