// Build-time generator of the filter-tap header used by the HIP kernels.
//
// Runs the library's own Daubechies derivation (hostmath.cpp) and writes the
// taps of db1..db8, rounded to float, as compile-time constants, so that the
// wavelet kernels carry them as instruction literals instead of registers.
//   usage: filtergen <output header>
#include <cstdio>
#include <vector>

#include "fhs_internal.h"

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: filtergen <header>\n");
    return 2;
  }
  FILE *f = std::fopen(argv[1], "w");
  if (!f) return 1;
  std::fprintf(f, "// Generated at build time by filtergen; do not edit.\n#pragma once\nnamespace fhs {\n");
  std::fprintf(f, "template <int NTAP> struct Taps;\n");
  for (int N = 1; N <= 8; ++N) {
    const std::vector<long double> h = fhs::daubechies(N);
    const int L = 2 * N;
    std::fprintf(f, "template <> struct Taps<%d> {\n  static constexpr float h[%d] = {", L, L);
    for (int m = 0; m < L; ++m) std::fprintf(f, "%s%.9ef", m ? ", " : "", static_cast<double>(static_cast<float>(h[m])));
    std::fprintf(f, "};\n  static constexpr float g[%d] = {", L);
    for (int m = 0; m < L; ++m) {
      const long double gm = ((m & 1) ? -1.0L : 1.0L) * h[L - 1 - m];
      std::fprintf(f, "%s%.9ef", m ? ", " : "", static_cast<double>(static_cast<float>(gm)));
    }
    std::fprintf(f, "};\n  static constexpr double hd[%d] = {", L);
    for (int m = 0; m < L; ++m) std::fprintf(f, "%s%.17e", m ? ", " : "", static_cast<double>(h[m]));
    std::fprintf(f, "};\n  static constexpr double gd[%d] = {", L);
    for (int m = 0; m < L; ++m) {
      const long double gm = ((m & 1) ? -1.0L : 1.0L) * h[L - 1 - m];
      std::fprintf(f, "%s%.17e", m ? ", " : "", static_cast<double>(gm));
    }
    std::fprintf(f, "};\n};\n");
  }
  std::fprintf(f, "}  // namespace fhs\n");
  std::fclose(f);
  return 0;
}
