// FP64 host arithmetic of the per-geometry plan (no device code).
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace bccb {

using cd = std::complex<double>;

// In-place radix-2 DFT of length n (power of two), sign -1 forward (unnormalised).
void host_dft(cd* x, int n, int sign);

// First column r of G = D_s^H D_s (property (iv) of Sec. III-A), grid [L2][L1]:
// r[l2][l1] = sum over kept (m1, m2) of e^{+j 2 pi (l1 m1 / L1 + l2 m2 / L2)}
// (the masked Kronecker sum of eq. (17) evaluated on its first column; each
// phase taken from the integer residue (l*m) mod L so no float product drifts).
std::vector<cd> gram_first_column(const uint8_t* mask, int M1, int M2, int L1, int L2);

// Omega[l2'][l1'] from eq. (21): lambda_{l2'} = F_L1( sum_{l2} r_{l2} e^{-j 2 pi l2 l2'/L2} ).
std::vector<cd> eigenvalues_eq21(const std::vector<cd>& r, int L1, int L2);

// e^{-j 2 pi j / N}, j < N, computed in FP64.
std::vector<cd> unit_roots(int N);

}  // namespace bccb
