// C entry points over the host embedding arithmetic (paper_2509_13592_amd/csrc/embed_math.cpp),
// built with g++ by tests/test_embed_math_cpu.py so the FP64 plan math of the padded-embedding
// plans can be checked against the oracle on the CPU.
#include <cstring>

#include "embed_math.h"

using namespace bccb;

extern "C" {

int em_embed_length(int L) { return embed_length(L); }

int em_spacing_fraction(double g, long* p, long* q) { return spacing_fraction(g, p, q) ? 1 : 0; }

double em_dirichlet_exact(long n, long N, int L) { return dirichlet_exact(n, N, L); }

void em_steering(int M, int L, double gamma, double* out) {
  const std::vector<cdx> W = steering_table(M, L, gamma);
  for (size_t i = 0; i < W.size(); ++i) {
    out[2 * i] = W[i].real();
    out[2 * i + 1] = W[i].imag();
  }
}

void em_toeplitz_spectrum(const uint8_t* mask, int M1, int M2, int L1, int L2, double g1, double g2, int P1, int P2,
                          double* out) {
  const std::vector<double> v = toeplitz_embedding_spectrum(mask, M1, M2, L1, L2, g1, g2, P1, P2);
  std::memcpy(out, v.data(), v.size() * sizeof(double));
}

void em_circulant_eigenvalues(const uint8_t* mask, int M1, int M2, int L1, int L2, double* out) {
  const std::vector<double> v = circulant_eigenvalues(mask, M1, M2, L1, L2);
  std::memcpy(out, v.data(), v.size() * sizeof(double));
}

void em_shifted_inverse_spectrum(const double* omega, int L1, int L2, double rho, int P1, int P2, double* out) {
  const std::vector<double> om(omega, omega + static_cast<size_t>(L1) * L2);
  const std::vector<double> v = shifted_inverse_embedding_spectrum(om, L1, L2, rho, P1, P2);
  std::memcpy(out, v.data(), v.size() * sizeof(double));
}

double em_gram_max_eigenvalue(const uint8_t* mask, int M1, int M2, int L1, int L2, double g1, double g2) {
  return gram_max_eigenvalue(mask, M1, M2, L1, L2, g1, g2);
}

}  // extern "C"
