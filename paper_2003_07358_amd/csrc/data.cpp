// The data-fidelity block: plan (uv-points, interpolation tables, scaling of
// Z, twiddles, inverse sampling density), workspace and the C ABI of the
// measurement operator and of the data dual update (Sec. 2.1 eq. model; Alg.
// 2 data-fidelity lines; Sec. 3.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>

#include "data_internal.h"
#include "fhs_internal.h"

using namespace fhs;
using namespace fhs::data;

namespace {

constexpr double kPi = 3.14159265358979323846;

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Kaiser-Bessel parameter for width J at oversampling alpha (Beatty, Nishimura
// and Pauly 2005) and the kernel psi(d) = I0(beta sqrt(1 - (2 d / J)^2)).
double kb_beta() {
  const double J = kKbWidth, a = kOversample;
  return kPi * std::sqrt((J / a) * (J / a) * (a - 0.5) * (a - 0.5) - 0.8);
}

double kb(double d, double beta) {
  const double J = kKbWidth;
  const double u = 1.0 - (2.0 * d / J) * (2.0 * d / J);
  if (u < 0.0) return 0.0;
  return std::cyl_bessel_i(0.0, beta * std::sqrt(u));
}

// Continuous Fourier transform of psi at xi (cycles per grid point):
// J sinh(r) / r with r = sqrt(beta^2 - (pi J xi)^2) (sin for imaginary r).
double kb_hat(double xi, double beta) {
  const double J = kKbWidth, q = beta * beta - (kPi * J * xi) * (kPi * J * xi);
  if (q > 0.0) {
    const double r = std::sqrt(q);
    return J * std::sinh(r) / r;
  }
  if (q < 0.0) {
    const double r = std::sqrt(-q);
    return J * std::sin(r) / r;
  }
  return J;
}

int check_data_plan(const fhs_data_plan *p) {
  if (!p) return fail(FHS_EINVAL, "null data plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_data_plan_set_workspace)");
  return FHS_OK;
}

template <typename T>
T *wsp(const fhs_data_plan *p, int64_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(p->ws) + off);
}

// x (image cube) -> Phi x (visibilities of every channel)
int forward(const fhs_data_plan *p, const float *x, float2v *vis, void *stream) {
  float2v *A = wsp<float2v>(p, p->off_a), *B = wsp<float2v>(p, p->off_b);
  PadArgs pa{x, A, wsp<float>(p, p->off_s1), wsp<float>(p, p->off_s2), p->ny, p->nx, p->L, p->K1, p->K2};
  if (int rc = launch_pad(pa, stream)) return rc;
  if (int rc = launch_fft_rows(A, static_cast<int64_t>(p->L) * p->K1, p->K2, wsp<float2v>(p, p->off_tw2), -1, stream))
    return rc;
  if (int rc = launch_transpose(A, B, p->K1, p->K2, p->L, stream)) return rc;
  if (int rc = launch_fft_rows(B, static_cast<int64_t>(p->L) * p->K2, p->K1, wsp<float2v>(p, p->off_tw1), -1, stream))
    return rc;
  InterpArgs ia{};
  ia.spec = B;
  ia.vis_out = vis;
  ia.info = wsp<VisInfo>(p, p->off_info);
  ia.w = wsp<float>(p, p->off_w);
  ia.perm = wsp<int32_t>(p, p->off_perm);
  ia.m = p->m;
  ia.K1 = p->K1;
  ia.K2 = p->K2;
  return launch_degrid(ia, stream);
}

// v (visibilities) -> x = beta x + scale_l Re(Phi^dagger v)
int adjoint(const fhs_data_plan *p, const float2v *vis, float *x, const double *scale, float beta, void *stream) {
  float2v *A = wsp<float2v>(p, p->off_a), *B = wsp<float2v>(p, p->off_b);
  const int64_t n = static_cast<int64_t>(p->L) * p->K1 * p->K2;
  if (int rc = launch_fill_zero(B, n, stream)) return rc;
  InterpArgs ia{};
  ia.grid = B;
  ia.vis_in = vis;
  ia.info = wsp<VisInfo>(p, p->off_info);
  ia.w = wsp<float>(p, p->off_w);
  ia.perm = wsp<int32_t>(p, p->off_perm);
  ia.items = wsp<GridItem>(p, p->off_items);
  ia.n_items = static_cast<int64_t>(p->items.size());
  ia.m = p->m;
  ia.K1 = p->K1;
  ia.K2 = p->K2;
  ia.wexp = p->wexp;
  if (int rc = launch_grid(ia, stream)) return rc;
  if (int rc = launch_fft_rows(B, static_cast<int64_t>(p->L) * p->K2, p->K1, wsp<float2v>(p, p->off_tw1), +1, stream))
    return rc;
  if (int rc = launch_transpose(B, A, p->K2, p->K1, p->L, stream)) return rc;
  if (int rc = launch_fft_rows(A, static_cast<int64_t>(p->L) * p->K1, p->K2, wsp<float2v>(p, p->off_tw2), +1, stream))
    return rc;
  CropArgs ca{A, x, wsp<float>(p, p->off_s1), wsp<float>(p, p->off_s2), scale, beta, p->ny, p->nx, p->L, p->K1, p->K2};
  return launch_crop(ca, stream);
}

}  // namespace

extern "C" {

int fhs_data_plan_create(const fhs_data_config *cfg, const int64_t *n_vis, const double *uv, fhs_data_plan **out) {
  if (!cfg || !n_vis || !uv || !out) return fail(FHS_EINVAL, "fhs_data_plan_create: null argument");
  *out = nullptr;
  const fhs_data_config c = *cfg;
  if (!pow2(c.ny) || !pow2(c.nx) || c.ny < 8 || c.nx < 8)
    return fail(FHS_EUNSUPPORTED, "the data block needs power-of-two image sides of at least 8 pixels");
  if (kOversample * c.ny > kMaxGrid || kOversample * c.nx > kMaxGrid)
    return fail(FHS_EUNSUPPORTED, "image side larger than 4096 pixels");
  if (c.nchan < 1) return fail(FHS_EINVAL, "need at least one channel");
  fhs_data_plan *p = new (std::nothrow) fhs_data_plan();
  if (!p) return fail(FHS_ENOMEM, "out of host memory");
  p->ny = c.ny;
  p->nx = c.nx;
  p->L = c.nchan;
  p->K1 = kOversample * c.ny;
  p->K2 = kOversample * c.nx;
  p->voff.assign(p->L + 1, 0);
  for (int l = 0; l < p->L; ++l) {
    if (n_vis[l] < 0) {
      delete p;
      return fail(FHS_EINVAL, "negative visibility count");
    }
    p->voff[l + 1] = p->voff[l] + n_vis[l];
  }
  p->m = p->voff[p->L];
  if (p->m >= (int64_t{1} << 31)) {
    delete p;
    return fail(FHS_EUNSUPPORTED, "more than 2^31 visibilities");
  }
  const double beta = kb_beta();
  // scaling of Z: 1 / psi^(m / K) at the centred pixel offsets m
  p->s1.resize(p->ny);
  p->s2.resize(p->nx);
  for (int n = 0; n < p->ny; ++n) p->s1[n] = static_cast<float>(1.0 / kb_hat((n - p->ny / 2) / double(p->K1), beta));
  for (int n = 0; n < p->nx; ++n) p->s2[n] = static_cast<float>(1.0 / kb_hat((n - p->nx / 2) / double(p->K2), beta));
  // twiddles exp(-2 pi i k / K), k < K / 2
  auto twiddles = [](int K, std::vector<float2v> &t) {
    t.resize(K / 2);
    for (int k = 0; k < K / 2; ++k) {
      const double a = -2.0 * kPi * k / K;
      t[k] = float2v{static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a))};
    }
  };
  twiddles(p->K1, p->tw1);
  twiddles(p->K2, p->tw2);
  // interpolation: grid coordinate t = omega K / (2 pi); the J points from
  // ceil(t - J / 2); inverse sampling density from the cell of the nearest
  // grid point
  p->info.resize(p->m);
  p->w.resize(p->m * 2 * kKbWidth);
  p->density_inv.resize(p->m);
  std::unordered_map<int64_t, int64_t> counts;
  std::vector<int64_t> cell(p->m);
  for (int l = 0; l < p->L; ++l)
    for (int64_t j = p->voff[l]; j < p->voff[l + 1]; ++j) {
      const double w1 = uv[2 * j], w2 = uv[2 * j + 1];
      if (!(std::fabs(w1) < 1e6) || !(std::fabs(w2) < 1e6)) {
        delete p;
        return fail(FHS_EINVAL, "uv-points must be finite, below 1e6 radians per pixel in magnitude");
      }
      const double t1 = w1 * p->K1 / (2.0 * kPi), t2 = w2 * p->K2 / (2.0 * kPi);
      const int64_t k1 = static_cast<int64_t>(std::ceil(t1 - kKbWidth / 2.0));
      const int64_t k2 = static_cast<int64_t>(std::ceil(t2 - kKbWidth / 2.0));
      VisInfo vi;
      vi.chan = l;
      vi.k1 = static_cast<int32_t>(((k1 % p->K1) + p->K1) % p->K1);
      vi.k2 = static_cast<int32_t>(((k2 % p->K2) + p->K2) % p->K2);
      vi.pad = 0;
      p->info[j] = vi;
      for (int a = 0; a < kKbWidth; ++a) {
        p->w[j * 2 * kKbWidth + a] = static_cast<float>(kb(t1 - static_cast<double>(k1 + a), beta));
        p->w[j * 2 * kKbWidth + kKbWidth + a] = static_cast<float>(kb(t2 - static_cast<double>(k2 + a), beta));
      }
      const int64_t c1 = ((static_cast<int64_t>(std::nearbyint(t1)) % p->K1) + p->K1) % p->K1;
      const int64_t c2 = ((static_cast<int64_t>(std::nearbyint(t2)) % p->K2) + p->K2) % p->K2;
      // (cells of different channels kept apart)
      cell[j] = (static_cast<int64_t>(l) * p->K1 + c1) * p->K2 + c2;
      ++counts[cell[j]];
    }
  for (int64_t j = 0; j < p->m; ++j) p->density_inv[j] = 1.0 / static_cast<double>(counts[cell[j]]);
  {
    // bound on the weight products, for the fixed-point gridding
    float wm = 0.0f;
    for (const float x : p->w) wm = std::max(wm, std::fabs(x));
    int e = 0;
    std::frexp(static_cast<double>(wm) * static_cast<double>(wm), &e);  // wm^2 < 2^e
    p->wexp = e;
  }
  // gridding order: visibilities sorted by (channel, tile of their first grid
  // indices), each run of one tile cut into work items of at most kGridChunk
  {
    const int64_t n2 = (p->K2 + kGridTile - 1) / kGridTile, n1 = (p->K1 + kGridTile - 1) / kGridTile;
    auto key = [&](int64_t j) {
      const VisInfo &v = p->info[j];
      return (static_cast<int64_t>(v.chan) * n1 + v.k1 / kGridTile) * n2 + v.k2 / kGridTile;
    };
    p->perm.resize(p->m);
    for (int64_t j = 0; j < p->m; ++j) p->perm[j] = static_cast<int32_t>(j);
    std::stable_sort(p->perm.begin(), p->perm.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
    for (int64_t i = 0; i < p->m;) {
      const int64_t k = key(p->perm[i]);
      int64_t e = i;
      while (e < p->m && key(p->perm[e]) == k) ++e;
      for (int64_t s0 = i; s0 < e; s0 += kGridChunk) {
        const VisInfo &v = p->info[p->perm[s0]];
        GridItem it{};
        it.chan = v.chan;
        it.t1 = v.k1 / kGridTile;
        it.t2 = v.k2 / kGridTile;
        it.start = static_cast<int32_t>(s0);
        it.count = static_cast<int32_t>(std::min<int64_t>(kGridChunk, e - s0));
        p->items.push_back(it);
      }
      i = e;
    }
  }
  // workspace: two grids, three visibility buffers, the tables
  const int64_t g = static_cast<int64_t>(p->L) * p->K1 * p->K2 * sizeof(float2v);
  const int64_t vb = std::max<int64_t>(p->m, 1) * sizeof(float2v);
  int64_t ws = 0;
  p->off_a = ws;
  ws = align256(ws + g);
  p->off_b = ws;
  ws = align256(ws + g);
  p->off_v1 = ws;
  ws = align256(ws + vb);
  p->off_v2 = ws;
  ws = align256(ws + vb);
  p->off_p = ws;
  ws = align256(ws + vb);
  p->off_info = ws;
  ws = align256(ws + std::max<int64_t>(p->m, 1) * sizeof(VisInfo));
  p->off_w = ws;
  ws = align256(ws + std::max<int64_t>(p->m, 1) * 2 * kKbWidth * sizeof(float));
  p->off_s1 = ws;
  ws = align256(ws + p->ny * sizeof(float));
  p->off_s2 = ws;
  ws = align256(ws + p->nx * sizeof(float));
  p->off_tw1 = ws;
  ws = align256(ws + (p->K1 / 2) * sizeof(float2v));
  p->off_tw2 = ws;
  ws = align256(ws + (p->K2 / 2) * sizeof(float2v));
  p->off_voff = ws;
  ws = align256(ws + (p->L + 1) * sizeof(int64_t));
  p->off_perm = ws;
  ws = align256(ws + std::max<int64_t>(p->m, 1) * sizeof(int32_t));
  p->off_items = ws;
  ws = align256(ws + std::max<int64_t>(static_cast<int64_t>(p->items.size()), 1) * sizeof(GridItem));
  p->off_part = ws;
  ws = align256(ws + static_cast<int64_t>(p->L) * kDualBlocks * 4 * sizeof(double));
  p->off_chs = ws;
  ws = align256(ws + static_cast<int64_t>(p->L) * 4 * sizeof(double));
  p->ws_bytes = ws;
  *out = p;
  return FHS_OK;
}

void fhs_data_plan_destroy(fhs_data_plan *plan) { delete plan; }

int fhs_data_plan_sizes(const fhs_data_plan *p, int64_t out[4]) {
  if (!p || !out) return fail(FHS_EINVAL, "fhs_data_plan_sizes: null argument");
  out[0] = p->m;
  out[1] = p->ws_bytes;
  out[2] = p->K1;
  out[3] = p->K2;
  return FHS_OK;
}

int fhs_data_plan_set_workspace(fhs_data_plan *p, void *dev_ptr, int64_t bytes) {
  if (!p) return fail(FHS_EINVAL, "fhs_data_plan_set_workspace: null plan");
  if (!dev_ptr || bytes < p->ws_bytes) return fail(FHS_EINVAL, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return fail(FHS_EINVAL, "workspace must be 256-byte aligned");
  char *b = static_cast<char *>(dev_ptr);
  auto up = [&](int64_t off, const void *src, size_t n) {
    return n == 0 || hipMemcpy(b + off, src, n, hipMemcpyHostToDevice) == hipSuccess;
  };
  const bool ok = up(p->off_info, p->info.data(), p->info.size() * sizeof(VisInfo)) &&
                  up(p->off_w, p->w.data(), p->w.size() * sizeof(float)) &&
                  up(p->off_s1, p->s1.data(), p->s1.size() * sizeof(float)) &&
                  up(p->off_s2, p->s2.data(), p->s2.size() * sizeof(float)) &&
                  up(p->off_tw1, p->tw1.data(), p->tw1.size() * sizeof(float2v)) &&
                  up(p->off_tw2, p->tw2.data(), p->tw2.size() * sizeof(float2v)) &&
                  up(p->off_voff, p->voff.data(), p->voff.size() * sizeof(int64_t)) &&
                  up(p->off_perm, p->perm.data(), p->perm.size() * sizeof(int32_t)) &&
                  up(p->off_items, p->items.data(), p->items.size() * sizeof(GridItem)) &&
                  hipDeviceSynchronize() == hipSuccess;
  if (!ok) return fail(FHS_EHIP, "fhs_data_plan_set_workspace: copying the tables failed");
  p->ws = dev_ptr;
  return FHS_OK;
}

int fhs_data_preconditioner(const fhs_data_plan *p, double *u) {
  if (!p || !u) return fail(FHS_EINVAL, "fhs_data_preconditioner: null argument");
  std::copy(p->density_inv.begin(), p->density_inv.end(), u);
  return FHS_OK;
}

int fhs_nufft_forward(const fhs_data_plan *p, const float *x, float *vis, void *stream) {
  if (int rc = check_data_plan(p)) return rc;
  if (!x || !vis) return fail(FHS_EINVAL, "fhs_nufft_forward: null array");
  return forward(p, x, reinterpret_cast<float2v *>(vis), stream);
}

int fhs_nufft_adjoint(const fhs_data_plan *p, const float *vis, float *x, const double *scale, float beta,
                      void *stream) {
  if (int rc = check_data_plan(p)) return rc;
  if (!x || !vis) return fail(FHS_EINVAL, "fhs_nufft_adjoint: null array");
  return adjoint(p, reinterpret_cast<const float2v *>(vis), x, scale, beta, stream);
}

int fhs_data_dual_update(const fhs_data_plan *p, const float *xcheck, const float *x, float *v, const float *y,
                         const float *U, const double *eps, const double *eta, int32_t n_sub, float *grad,
                         double *residual, void *stream) {
  if (int rc = check_data_plan(p)) return rc;
  if (!xcheck || !x || !v || !y || !U || !eps || !eta || !grad)
    return fail(FHS_EINVAL, "fhs_data_dual_update: null array");
  if (n_sub < 0) return fail(FHS_EINVAL, "n_sub must be >= 0");
  float2v *yc = wsp<float2v>(p, p->off_v1), *yx = wsp<float2v>(p, p->off_v2);
  if (int rc = forward(p, xcheck, yc, stream)) return rc;
  if (int rc = forward(p, x, yx, stream)) return rc;
  DualArgs d{};
  d.yc = yc;
  d.yx = yx;
  d.v = reinterpret_cast<float2v *>(v);
  d.y = reinterpret_cast<const float2v *>(y);
  d.U = U;
  d.p = wsp<float2v>(p, p->off_p);
  d.eps = eps;
  d.voff = wsp<int64_t>(p, p->off_voff);
  d.residual = residual;
  d.part = wsp<double>(p, p->off_part);
  d.chs = wsp<double>(p, p->off_chs);
  d.n_sub = n_sub;
  d.L = p->L;
  if (int rc = launch_data_dual(d, stream)) return rc;
  return adjoint(p, reinterpret_cast<const float2v *>(v), grad, eta, 1.0f, stream);
}

}  // extern "C"
