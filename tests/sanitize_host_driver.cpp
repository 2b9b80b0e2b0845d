// Host-side driver for the sanitizer test (tests/test_host_sanitize_cpu.py):
// plan creation, queries and destruction of the library's plan code, built
// with AddressSanitizer and UndefinedBehaviorSanitizer and run without a GPU.
// The device launchers of the data block are never reached here (no workspace
// is attached); they are defined as failing stand-ins so that the host files
// link on their own.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "data_internal.h"
#include "fhs.h"
#include "fhs_internal.h"

namespace fhs {
namespace data {
int launch_pad(const PadArgs &, void *) { return FHS_EHIP; }
int launch_crop(const CropArgs &, void *) { return FHS_EHIP; }
int launch_fft_rows(float2v *, int64_t, int, const float2v *, int, void *) { return FHS_EHIP; }
int launch_transpose(const float2v *, float2v *, int, int, int, void *) { return FHS_EHIP; }
int launch_fill_zero(float2v *, int64_t, void *) { return FHS_EHIP; }
int launch_degrid(const InterpArgs &, void *) { return FHS_EHIP; }
int launch_grid(const InterpArgs &, void *) { return FHS_EHIP; }
int launch_data_dual(const DualArgs &, void *) { return FHS_EHIP; }
}  // namespace data
void prof_release(fhs_plan *) {}
}  // namespace fhs

static int failures = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                 \
    }                                                             \
  } while (0)

static void exercise(const fhs_config &c, bool valid) {
  fhs_plan *p = nullptr;
  const int rc = fhs_plan_create(&c, &p);
  CHECK((rc == FHS_OK) == valid);
  if (rc != FHS_OK) {
    CHECK(p == nullptr);
    return;
  }
  fhs_sizes s{};
  CHECK(fhs_plan_sizes(p, &s) == FHS_OK);
  int64_t f[12];
  for (int64_t i = 0; i < s.n_facets; ++i) CHECK(fhs_plan_facet(p, static_cast<int32_t>(i), f) == FHS_OK);
  CHECK(fhs_plan_facet(p, static_cast<int32_t>(s.n_facets), f) != FHS_OK);
  int64_t b[4];
  for (int64_t i = 0; i < s.n_bands; ++i) CHECK(fhs_plan_band(p, static_cast<int32_t>(i), b) == FHS_OK);
  std::vector<double> sb(c.n_sub, 0.1), mu(c.n_sub), mub(s.n_facets);
  CHECK(fhs_plan_heuristics(p, sb.data(), mu.data(), mub.data()) == FHS_OK);
  fhs_tuning t{};
  CHECK(fhs_plan_get_tuning(p, &t) == FHS_OK);
  CHECK(fhs_plan_set_tuning(p, &t) == FHS_OK);
  t.nuc_seg = 7;
  CHECK(fhs_plan_set_tuning(p, &t) != FHS_OK);
  fhs_plan_destroy(p);
}

int main() {
  //                  ny    nx   L  qy qx  C  oy  ox lev prec spec
  exercise(fhs_config{256, 256, 20, 2, 2, 1, 32, 32, 4, 0, 0}, true);
  exercise(fhs_config{101, 77, 6, 3, 2, 2, 7, 5, 3, 0, 0}, true);
  exercise(fhs_config{7, 9, 3, 1, 1, 1, 0, 0, 2, 0, 0}, true);
  exercise(fhs_config{64, 64, 100, 2, 2, 10, 8, 8, 2, 0, 2}, true);
  exercise(fhs_config{64, 64, 12, 4, 4, 4, 0, 0, 6, 1, 0}, true);
  exercise(fhs_config{300, 260, 8, 64, 64, 1, 2, 2, 1, 0, 0}, true);
  exercise(fhs_config{64, 64, 8, 2, 2, 3, 8, 8, 4, 0, 0}, false);   // C does not divide L
  exercise(fhs_config{64, 64, 8, 2, 2, 1, 40, 8, 4, 0, 0}, false);  // overlap larger than a tile
  exercise(fhs_config{64, 64, 8, 1, 1, 2, 0, 0, 4, 0, 9}, false);   // overlap wider than a block
  exercise(fhs_config{64, 64, 8, 1, 1, 1, 0, 0, 7, 0, 0}, false);   // levels
  exercise(fhs_config{64, 64, 130, 1, 1, 1, 0, 0, 4, 0, 0}, false); // channels per sub-cube
  // the data plan: tables, density, sizes; invalid sides and points
  {
    const int L = 3;
    std::vector<int64_t> n{500, 0, 37};
    std::vector<double> uv;
    unsigned seed = 12345u;
    for (int64_t j = 0; j < 537; ++j)
      for (int k = 0; k < 2; ++k) {
        seed = seed * 1664525u + 1013904223u;
        uv.push_back((seed / 4294967296.0 - 0.5) * 7.0);
      }
    fhs_data_config dc{32, 64, L};
    fhs_data_plan *d = nullptr;
    CHECK(fhs_data_plan_create(&dc, n.data(), uv.data(), &d) == FHS_OK);
    int64_t sz[4];
    CHECK(fhs_data_plan_sizes(d, sz) == FHS_OK && sz[0] == 537 && sz[2] == 64 && sz[3] == 128);
    std::vector<double> u(537);
    CHECK(fhs_data_preconditioner(d, u.data()) == FHS_OK);
    for (double v : u) CHECK(v > 0.0 && v <= 1.0);
    CHECK(fhs_nufft_forward(d, nullptr, nullptr, nullptr) != FHS_OK);  // no workspace
    fhs_data_plan_destroy(d);
    fhs_data_config bad{48, 64, L};
    d = nullptr;
    CHECK(fhs_data_plan_create(&bad, n.data(), uv.data(), &d) != FHS_OK && d == nullptr);
    uv[5] = 1e300;
    CHECK(fhs_data_plan_create(&dc, n.data(), uv.data(), &d) != FHS_OK && d == nullptr);
  }
  std::printf("sanitized host checks: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
