// Host-side mathematics of libfhs: Daubechies filters and chi moments.
//
// Filters.  The SARA dictionary uses the first eight Daubechies wavelets
// (Sec. 2.3.1).  dbN is built from Daubechies' 1988 construction: the squared
// modulus of the low-pass transfer function is cos^{2N}(w/2) P(sin^2(w/2)),
// P(y) = sum_{k<N} binom(N-1+k, k) y^k.  The N-1 roots of P are found with the
// Durand-Kerner (Weierstrass) simultaneous iteration in long double; each
// root y_k gives the pair r, 1/r of z^2 - (2 - 4 y_k) z + 1 and the root outside
// the unit circle is kept (extremal phase, energy at the start of the
// filter).  h[n] = sqrt(2) [z^n] ((1+z)/2)^N prod_k (z - r_k) / (1 - r_k).
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

#include "fhs_internal.h"

namespace fhs {

using cld = std::complex<long double>;

static std::vector<cld> durand_kerner(const std::vector<long double> &a_asc) {
  // roots of sum_k a_k y^k (degree n = size-1)
  const int n = static_cast<int>(a_asc.size()) - 1;
  std::vector<cld> r(n);
  if (n <= 0) return r;
  const long double lead = a_asc[n];
  const cld seed(0.4L, 0.9L);
  cld cur(1.0L, 0.0L);
  for (int i = 0; i < n; ++i) {
    r[i] = cur;
    cur *= seed;
  }
  auto eval = [&](cld y) {
    cld v(0.0L, 0.0L);
    for (int k = n; k >= 0; --k) v = v * y + cld(a_asc[k] / lead, 0.0L);
    return v;
  };
  for (int it = 0; it < 2000; ++it) {
    long double change = 0.0L;
    for (int i = 0; i < n; ++i) {
      cld den(1.0L, 0.0L);
      for (int j = 0; j < n; ++j)
        if (j != i) den *= (r[i] - r[j]);
      const cld d = eval(r[i]) / den;
      r[i] -= d;
      change = std::max(change, std::abs(d));
    }
    if (change < 1e-30L) break;
  }
  return r;
}

std::vector<long double> daubechies(int N) {
  if (N < 1 || N > 20) throw std::invalid_argument("dbN: N out of range");
  std::vector<long double> p(N);
  for (int k = 0; k < N; ++k) {
    // binom(N-1+k, k)
    long double b = 1.0L;
    for (int i = 1; i <= k; ++i) b = b * static_cast<long double>(N - 1 + i) / static_cast<long double>(i);
    p[k] = b;
  }
  std::vector<cld> yr = durand_kerner(p);
  // ascending coefficients of the polynomial in z
  std::vector<cld> poly{cld(1.0L, 0.0L)};
  auto mul_linear = [&](cld c0, cld c1) {  // poly *= (c0 + c1 z)
    std::vector<cld> out(poly.size() + 1, cld(0.0L, 0.0L));
    for (size_t i = 0; i < poly.size(); ++i) {
      out[i] += poly[i] * c0;
      out[i + 1] += poly[i] * c1;
    }
    poly.swap(out);
  };
  for (int i = 0; i < N; ++i) mul_linear(cld(0.5L, 0.0L), cld(0.5L, 0.0L));
  for (const cld &y : yr) {
    const cld b = cld(2.0L, 0.0L) - cld(4.0L, 0.0L) * y;
    const cld disc = std::sqrt(b * b - cld(4.0L, 0.0L));
    cld z = (b + disc) / cld(2.0L, 0.0L);
    if (std::abs(z) <= 1.0L) z = (b - disc) / cld(2.0L, 0.0L);
    const cld norm = cld(1.0L, 0.0L) / (cld(1.0L, 0.0L) - z);
    mul_linear(-z * norm, norm);
  }
  std::vector<long double> h(2 * N);
  const long double s2 = std::sqrt(2.0L);
  for (int n = 0; n < 2 * N; ++n) h[n] = s2 * poly[n].real();
  return h;
}

void chi_mean_std(double k, double *m, double *s) {
  const double mean = std::sqrt(2.0) * std::exp(std::lgamma((k + 1.0) / 2.0) - std::lgamma(k / 2.0));
  *m = mean;
  *s = std::sqrt(std::max(0.0, k - mean * mean));
}

}  // namespace fhs
