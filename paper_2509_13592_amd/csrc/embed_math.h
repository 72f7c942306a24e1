// FP64 host arithmetic of plans on a zero-padded circulant embedding (no device code):
// uniform harmonic grids at a general element spacing gamma_i (Toeplitz Gram, Sec. III-A
// with eq. (16)) and grid lengths that are not powers of two.
//
// On the grid f_{i,l} = -gamma_i + l 2 gamma_i / L_i the Gram D_s^H D_s is block Toeplitz
// with Toeplitz blocks: G[(l1, l2), (l1', l2')] = t(l1 - l1', l2 - l2') with
//   t(d1, d2) = sum over kept (m1, m2) of e^{+j 2 pi (2 gamma1 d1 m1 / L1 + 2 gamma2 d2 m2 / L2)}
// (the masked Kronecker sum of eq. (17)), |d_i| < L_i.  Placing t(d) at index d mod P_i of a
// P1 x P2 grid, P_i >= 2 L_i - 1, gives the first column of a BCCB whose leading L1 x L2
// window is G; its eigenvalues (eq. (21) applied to that column) are what the passes
// multiply by, with the iterate held at zero outside the window.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace bccb {

using cdx = std::complex<double>;

// Transform length of the embedding: the smallest power of two >= max(8, 2 L - 1).
int embed_length(int L);

// gamma = p / q with q <= 4096 when the double is exactly that fraction (true), else false.
bool spacing_fraction(double gamma, long* p, long* q);

// Steering table W[m * L + l] = e^{-j 2 pi f_l m}, m < M, l < L, on the grid
// f_l = -gamma + l 2 gamma / L (eqs. (5), (16)); phases from integer residues when gamma
// is a fraction p/q (f_l m = p m (2 l - L) / (q L)).
std::vector<cdx> steering_table(int M, int L, double gamma);

// sum_{d = -(L-1)}^{L-1} e^{j 2 pi d n / N} for integers n, N > 0 (a real Dirichlet sum).
double dirichlet_exact(long n, long N, int L);
// the same sum at a real frequency x (cycles per sample): sum_{|d| < L} e^{j 2 pi d x}.
double dirichlet_real(double x, int L);

// Eigenvalues Omega_e[q2 * P1 + q1] of the embedding of the Gram (real: t(-d) = conj t(d)).
std::vector<double> toeplitz_embedding_spectrum(const uint8_t* mask, int M1, int M2, int L1, int L2,
                                                double gamma1, double gamma2, int P1, int P2);

// Eigenvalues of the L1 x L2 BCCB Gram at gamma = 1/2 (eq. (21)): L1 L2 times the number of
// kept elements folding onto each bin, omega[k2 * L1 + k1].
std::vector<double> circulant_eigenvalues(const uint8_t* mask, int M1, int M2, int L1, int L2);

// Eigenvalues of the embedding of (G + rho I)^-1 for the BCCB G of the eigenvalue grid `omega`
// (L1 x L2): 1/rho + (1 / (L1 L2)) sum over bins k with omega_k != 0 of
// (1/(omega_k + rho) - 1/rho) D_{L1}(k1 P1 - q1 L1, L1 P1) D_{L2}(k2 P2 - q2 L2, L2 P2).
std::vector<double> shifted_inverse_embedding_spectrum(const std::vector<double>& omega, int L1, int L2,
                                                       double rho, int P1, int P2);

// Largest eigenvalue of D_s D_s^H (= sigma_max(D_s)^2, the inverse step of eq. (9)) on the
// spaced grid, by Lanczos with full reorthogonalisation (min(M, 320) steps) and bisection on
// the tridiagonal matrix.
double gram_max_eigenvalue(const uint8_t* mask, int M1, int M2, int L1, int L2, double gamma1, double gamma2);

}  // namespace bccb
