// FP64 host arithmetic of plans on a zero-padded circulant embedding (declarations and the
// derivation in embed_math.h).
#include "embed_math.h"

#include <algorithm>
#include <cmath>

namespace bccb {

namespace {
constexpr double kPi = 3.14159265358979323846264338327950288;

long mod_pos(long a, long n) {
  const long r = a % n;
  return r < 0 ? r + n : r;
}

// e^{-j 2 pi n / N}
cdx unit(long n, long N) {
  const double a = -2.0 * kPi * static_cast<double>(mod_pos(n, N)) / static_cast<double>(N);
  return cdx(std::cos(a), std::sin(a));
}
}  // namespace

int embed_length(int L) {
  int P = 8;
  while (P < 2 * L - 1) P <<= 1;
  return P;
}

bool spacing_fraction(double gamma, long* p, long* q) {
  if (!(gamma > 0.0) || !std::isfinite(gamma)) return false;
  // continued-fraction convergents of gamma; the first whose quotient is gamma exactly wins
  long h0 = 0, h1 = 1, k0 = 1, k1 = 0;
  double x = gamma;
  for (int it = 0; it < 40; ++it) {
    const double a = std::floor(x);
    if (a > 1e9) break;
    const long ai = static_cast<long>(a);
    const long h2 = ai * h1 + h0, k2 = ai * k1 + k0;
    if (k2 > 4096) break;
    if (static_cast<double>(h2) / static_cast<double>(k2) == gamma) {
      *p = h2;
      *q = k2;
      return true;
    }
    h0 = h1;
    h1 = h2;
    k0 = k1;
    k1 = k2;
    const double frac = x - a;
    if (frac <= 0.0) break;
    x = 1.0 / frac;
  }
  return false;
}

std::vector<cdx> steering_table(int M, int L, double gamma) {
  std::vector<cdx> W(static_cast<size_t>(M) * L);
  long p = 0, q = 0;
  const bool exact = spacing_fraction(gamma, &p, &q);
  for (int m = 0; m < M; ++m) {
    for (int l = 0; l < L; ++l) {
      cdx w;
      if (exact) {
        w = unit(p * m * (2L * l - L), q * L);   // f_l m = p m (2 l - L) / (q L)
      } else {
        const double ph = (-gamma + 2.0 * gamma * l / L) * m;
        const double r = ph - std::floor(ph);
        w = cdx(std::cos(-2.0 * kPi * r), std::sin(-2.0 * kPi * r));
      }
      W[static_cast<size_t>(m) * L + l] = w;
    }
  }
  return W;
}

double dirichlet_exact(long n, long N, int L) {
  const long r = mod_pos(n, N);
  if (r == 0) return 2.0 * L - 1.0;
  // sin(pi (2L - 1) n / N) / sin(pi n / N); both phases reduced as integers mod 2N
  const long num = mod_pos(static_cast<long>(2 * L - 1) * r, 2 * N);
  return std::sin(kPi * static_cast<double>(num) / static_cast<double>(N)) /
         std::sin(kPi * static_cast<double>(r) / static_cast<double>(N));
}

double dirichlet_real(double x, int L) {
  const double e = x - std::round(x);   // the sum has period 1 in x
  if (std::fabs(e) < 1e-13) return 2.0 * L - 1.0;
  return std::sin(kPi * (2.0 * L - 1.0) * e) / std::sin(kPi * e);
}

// F[m * P + q] = sum_{|d| < L} e^{j 2 pi d (2 gamma m / L - q / P)}: the DFT over the
// embedding of one kept element's Toeplitz factor along one axis.
static std::vector<double> axis_factor(int M, int L, double gamma, int P) {
  std::vector<double> F(static_cast<size_t>(M) * P);
  long p = 0, q = 0;
  const bool exact = spacing_fraction(gamma, &p, &q);
  for (int m = 0; m < M; ++m) {
    for (int k = 0; k < P; ++k) {
      double v;
      if (exact) {
        // 2 gamma m / L - k / P = (2 p m P - k q L) / (q L P)
        v = dirichlet_exact(2 * p * m * static_cast<long>(P) - static_cast<long>(k) * q * L,
                            q * static_cast<long>(L) * P, L);
      } else {
        v = dirichlet_real(2.0 * gamma * m / L - static_cast<double>(k) / P, L);
      }
      F[static_cast<size_t>(m) * P + k] = v;
    }
  }
  return F;
}

std::vector<double> toeplitz_embedding_spectrum(const uint8_t* mask, int M1, int M2, int L1, int L2,
                                                double gamma1, double gamma2, int P1, int P2) {
  const std::vector<double> F1 = axis_factor(M1, L1, gamma1, P1);
  const std::vector<double> F2 = axis_factor(M2, L2, gamma2, P2);
  std::vector<double> om(static_cast<size_t>(P1) * P2, 0.0);
  std::vector<double> row(P1);
  for (int m2 = 0; m2 < M2; ++m2) {
    std::fill(row.begin(), row.end(), 0.0);
    bool any = false;
    for (int m1 = 0; m1 < M1; ++m1) {
      if (!mask[static_cast<size_t>(m2) * M1 + m1]) continue;
      any = true;
      const double* f1 = &F1[static_cast<size_t>(m1) * P1];
      for (int q1 = 0; q1 < P1; ++q1) row[q1] += f1[q1];
    }
    if (!any) continue;
    const double* f2 = &F2[static_cast<size_t>(m2) * P2];
    for (int q2 = 0; q2 < P2; ++q2) {
      double* o = &om[static_cast<size_t>(q2) * P1];
      for (int q1 = 0; q1 < P1; ++q1) o[q1] += f2[q2] * row[q1];
    }
  }
  return om;
}

std::vector<double> circulant_eigenvalues(const uint8_t* mask, int M1, int M2, int L1, int L2) {
  std::vector<double> om(static_cast<size_t>(L1) * L2, 0.0);
  const double L = static_cast<double>(L1) * L2;
  for (int m2 = 0; m2 < M2; ++m2)
    for (int m1 = 0; m1 < M1; ++m1)
      if (mask[static_cast<size_t>(m2) * M1 + m1]) om[static_cast<size_t>(m2 % L2) * L1 + (m1 % L1)] += L;
  return om;
}

std::vector<double> shifted_inverse_embedding_spectrum(const std::vector<double>& omega, int L1, int L2,
                                                       double rho, int P1, int P2) {
  std::vector<double> out(static_cast<size_t>(P1) * P2, 1.0 / rho);
  const double invL = 1.0 / (static_cast<double>(L1) * L2);
  std::vector<double> row(P1);
  for (int k2 = 0; k2 < L2; ++k2) {
    std::fill(row.begin(), row.end(), 0.0);
    bool any = false;
    for (int k1 = 0; k1 < L1; ++k1) {
      const double w = omega[static_cast<size_t>(k2) * L1 + k1];
      if (w == 0.0) continue;
      any = true;
      const double s = (1.0 / (w + rho) - 1.0 / rho) * invL;
      for (int q1 = 0; q1 < P1; ++q1)
        row[q1] += s * dirichlet_exact(static_cast<long>(k1) * P1 - static_cast<long>(q1) * L1,
                                       static_cast<long>(L1) * P1, L1);
    }
    if (!any) continue;
    for (int q2 = 0; q2 < P2; ++q2) {
      const double d2 = dirichlet_exact(static_cast<long>(k2) * P2 - static_cast<long>(q2) * L2,
                                        static_cast<long>(L2) * P2, L2);
      double* o = &out[static_cast<size_t>(q2) * P1];
      for (int q1 = 0; q1 < P1; ++q1) o[q1] += d2 * row[q1];
    }
  }
  return out;
}

// A_i(delta) = sum_{l < L} e^{-j 2 pi f_l delta}, delta = -(M-1) .. M-1, stored at delta + M - 1.
static std::vector<cdx> axis_outer(int M, int L, double gamma) {
  std::vector<cdx> A(2 * static_cast<size_t>(M) - 1, cdx(0, 0));
  long p = 0, q = 0;
  const bool exact = spacing_fraction(gamma, &p, &q);
  for (int dl = -(M - 1); dl <= M - 1; ++dl) {
    cdx s(0, 0);
    for (int l = 0; l < L; ++l) {
      if (exact) {
        s += unit(p * static_cast<long>(dl) * (2L * l - L), q * L);
      } else {
        const double ph = (-gamma + 2.0 * gamma * l / L) * dl;
        const double r = ph - std::floor(ph);
        s += cdx(std::cos(-2.0 * kPi * r), std::sin(-2.0 * kPi * r));
      }
    }
    A[static_cast<size_t>(dl + M - 1)] = s;
  }
  return A;
}

// Largest eigenvalue of the symmetric tridiagonal matrix (a, b) by bisection on Sturm counts.
static double tridiag_max_eigenvalue(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = static_cast<int>(a.size());
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  // count of eigenvalues below x
  auto below = [&](double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
      const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = a[i] - x - (i > 0 ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= n) hi = mid;   // every eigenvalue lies below mid
    else lo = mid;
  }
  return hi;
}

double gram_max_eigenvalue(const uint8_t* mask, int M1, int M2, int L1, int L2, double gamma1, double gamma2) {
  std::vector<int> s1, s2;
  for (int m2 = 0; m2 < M2; ++m2)
    for (int m1 = 0; m1 < M1; ++m1)
      if (mask[static_cast<size_t>(m2) * M1 + m1]) {
        s1.push_back(m1);
        s2.push_back(m2);
      }
  const int M = static_cast<int>(s1.size());
  if (M == 0) return 0.0;
  const std::vector<cdx> A1 = axis_outer(M1, L1, gamma1), A2 = axis_outer(M2, L2, gamma2);
  // K = D_s D_s^H, K[m][m'] = A1(m1 - m1') A2(m2 - m2') (the separable Gram of the rows)
  std::vector<cdx> K(static_cast<size_t>(M) * M);
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j)
      K[static_cast<size_t>(i) * M + j] = A1[static_cast<size_t>(s1[i] - s1[j] + M1 - 1)] *
                                          A2[static_cast<size_t>(s2[i] - s2[j] + M2 - 1)];
  const int steps = std::min(M, 320);
  std::vector<std::vector<cdx>> V;
  V.reserve(steps);
  std::vector<cdx> v(M);
  double nv = 0.0;
  for (int i = 0; i < M; ++i) {
    v[i] = cdx(1.0 + 0.37 * std::sin(1.0 + 2.3 * i), 0.21 * std::cos(0.7 + 1.9 * i));
    nv += std::norm(v[i]);
  }
  nv = std::sqrt(nv);
  for (cdx& x : v) x /= nv;
  std::vector<double> alpha, beta;
  std::vector<cdx> w(M);
  for (int k = 0; k < steps; ++k) {
    V.push_back(v);
    for (int i = 0; i < M; ++i) {
      cdx acc(0, 0);
      const cdx* kr = &K[static_cast<size_t>(i) * M];
      for (int j = 0; j < M; ++j) acc += kr[j] * v[j];
      w[i] = acc;
    }
    double a = 0.0;
    for (int i = 0; i < M; ++i) a += std::real(std::conj(v[i]) * w[i]);
    alpha.push_back(a);
    // full reorthogonalisation (twice) against every Lanczos vector so far
    for (int pass = 0; pass < 2; ++pass) {
      for (const auto& u : V) {
        cdx c(0, 0);
        for (int i = 0; i < M; ++i) c += std::conj(u[i]) * w[i];
        for (int i = 0; i < M; ++i) w[i] -= c * u[i];
      }
    }
    double bn = 0.0;
    for (int i = 0; i < M; ++i) bn += std::norm(w[i]);
    bn = std::sqrt(bn);
    if (k + 1 == steps || bn <= 1e-12 * std::fabs(a) + 1e-300) break;
    beta.push_back(bn);
    for (int i = 0; i < M; ++i) v[i] = w[i] / bn;
  }
  beta.resize(alpha.size() > 0 ? alpha.size() - 1 : 0);
  return tridiag_max_eigenvalue(alpha, beta);
}

}  // namespace bccb
