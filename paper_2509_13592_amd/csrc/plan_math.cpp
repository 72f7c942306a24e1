// FP64 host arithmetic of the per-geometry plan: first column of the Gram and
// its BCCB eigenvalues (Sec. III-A property (iv), eq. (17), eq. (21)).
#include "plan_math.h"

#include <cmath>

namespace bccb {

namespace {
constexpr double kTwoPi = 6.283185307179586476925286766559;
}

std::vector<cd> unit_roots(int N) {
  std::vector<cd> w(N);
  for (int j = 0; j < N; ++j) {
    const double a = -kTwoPi * static_cast<double>(j) / static_cast<double>(N);
    w[j] = cd(std::cos(a), std::sin(a));
  }
  return w;
}

void host_dft(cd* x, int n, int sign) {
  // bit-reversal permutation
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  const std::vector<cd> w = unit_roots(n);
  for (int len = 2; len <= n; len <<= 1) {
    const int step = n / len;
    for (int i = 0; i < n; i += len) {
      for (int k = 0; k < len / 2; ++k) {
        cd tw = w[k * step];
        if (sign > 0) tw = std::conj(tw);
        const cd a = x[i + k];
        const cd b = x[i + k + len / 2] * tw;
        x[i + k] = a + b;
        x[i + k + len / 2] = a - b;
      }
    }
  }
}

std::vector<cd> gram_first_column(const uint8_t* mask, int M1, int M2, int L1, int L2) {
  // e^{+j 2 pi k / L} tables
  std::vector<cd> e1 = unit_roots(L1), e2 = unit_roots(L2);
  for (cd& v : e1) v = std::conj(v);
  for (cd& v : e2) v = std::conj(v);
  // P[m2][l1] = sum over kept m1 in row m2 of e^{+j 2 pi l1 m1 / L1}
  std::vector<cd> P(static_cast<size_t>(M2) * L1, cd(0, 0));
  for (int m2 = 0; m2 < M2; ++m2) {
    for (int m1 = 0; m1 < M1; ++m1) {
      if (!mask[static_cast<size_t>(m2) * M1 + m1]) continue;
      for (int l1 = 0; l1 < L1; ++l1)
        P[static_cast<size_t>(m2) * L1 + l1] += e1[(static_cast<long>(l1) * m1) % L1];
    }
  }
  // r[l2][l1] = sum_{m2} e^{+j 2 pi l2 m2 / L2} P[m2][l1]
  std::vector<cd> r(static_cast<size_t>(L1) * L2, cd(0, 0));
  for (int m2 = 0; m2 < M2; ++m2) {
    bool any = false;
    for (int m1 = 0; m1 < M1 && !any; ++m1) any = mask[static_cast<size_t>(m2) * M1 + m1] != 0;
    if (!any) continue;
    for (int l2 = 0; l2 < L2; ++l2) {
      const cd ph = e2[(static_cast<long>(l2) * m2) % L2];
      cd* rr = &r[static_cast<size_t>(l2) * L1];
      const cd* pp = &P[static_cast<size_t>(m2) * L1];
      for (int l1 = 0; l1 < L1; ++l1) rr[l1] += ph * pp[l1];
    }
  }
  return r;
}

std::vector<cd> eigenvalues_eq21(const std::vector<cd>& r, int L1, int L2) {
  std::vector<cd> om(r);
  // L2-point DFT of the block sequence {r_l2}, element-wise over l1
  std::vector<cd> col(L2);
  for (int l1 = 0; l1 < L1; ++l1) {
    for (int l2 = 0; l2 < L2; ++l2) col[l2] = om[static_cast<size_t>(l2) * L1 + l1];
    host_dft(col.data(), L2, -1);
    for (int l2 = 0; l2 < L2; ++l2) om[static_cast<size_t>(l2) * L1 + l1] = col[l2];
  }
  // F_L1 of each lambda_{l2'}
  for (int l2 = 0; l2 < L2; ++l2) host_dft(&om[static_cast<size_t>(l2) * L1], L1, -1);
  return om;
}

}  // namespace bccb
