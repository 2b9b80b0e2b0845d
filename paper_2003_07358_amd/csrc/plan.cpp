// Plan creation and host-only ABI entry points of libfhs.
//
// Geometry (Sec. 2.4.2): tiles t_s = floor(s n / Q) per axis; the low-rankness
// facet of tile s extends `overlap` pixels toward the top/left except on the
// first row/column of tiles, where it keeps the tile size; the apodisation
// window D_q is evaluated on the fly by the kernels from these bounds.
// Wavelet bands: zero-extended expansive transform, K = floor((n + L - 1) / 2)
// coefficients per band and level for an input of n samples and L taps.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include <hip/hip_runtime.h>

#include "fhs_internal.h"

namespace fhs {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

static int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

}  // namespace fhs

namespace fhs {
int64_t nuc_recon_lds(const fhs_plan *p, int S) {
  const int64_t W = p->lc16;
  if (p->C == 1) return (4 * static_cast<int64_t>(S) * p->L + 64) * 4;  // K held in registers
  // K matrices, two staging buffers of X [S][L] and P [C][S][Ln], the output tile [C][S][Ln]
  return static_cast<int64_t>(p->C) * W * (W + 1) * 8 +
         static_cast<int64_t>(S) * (2 * p->L + 3 * static_cast<int64_t>(p->C) * p->Ln) * 4;
}
}  // namespace fhs

using namespace fhs;

extern "C" {

int fhs_version(void) { return 200; }

const char *fhs_last_error(void) { return g_err.c_str(); }

int fhs_filter(int32_t N, double *h_out) {
  if (N < 1 || N > 8 || !h_out) return fail(FHS_EINVAL, "fhs_filter: N must be in 1..8 and h_out non-null");
  try {
    std::vector<long double> h = daubechies(N);
    for (int i = 0; i < 2 * N; ++i) h_out[i] = static_cast<double>(h[i]);
  } catch (const std::exception &e) {
    return fail(FHS_EINVAL, e.what());
  }
  return FHS_OK;
}

int fhs_chi_mean_std(double k, double *mean, double *std_dev) {
  if (!(k > 0) || !mean || !std_dev) return fail(FHS_EINVAL, "fhs_chi_mean_std: k > 0 and non-null outputs required");
  chi_mean_std(k, mean, std_dev);
  return FHS_OK;
}

int fhs_plan_create(const fhs_config *cfg, fhs_plan **out) {
  if (!cfg || !out) return fail(FHS_EINVAL, "fhs_plan_create: null argument");
  *out = nullptr;
  const fhs_config c = *cfg;
  if (c.ny < 1 || c.nx < 1 || c.nchan < 1) return fail(FHS_EINVAL, "image and channel sizes must be positive");
  if (c.qy < 1 || c.qx < 1 || c.qy > kMaxFacetAxis || c.qx > kMaxFacetAxis)
    return fail(FHS_EINVAL, "facets per axis must be in 1..64");
  if (c.qy > c.ny || c.qx > c.nx) return fail(FHS_EINVAL, "more facets than pixels along an axis");
  if (c.n_sub < 1 || c.nchan % c.n_sub != 0)
    return fail(FHS_EUNSUPPORTED, "the number of sub-cubes must divide the number of channels");
  if (c.nchan / c.n_sub > kMaxLc) return fail(FHS_EUNSUPPORTED, "more than 64 channels per sub-cube");
  if (c.overlap_y < 0 || c.overlap_x < 0) return fail(FHS_EINVAL, "negative overlap");
  if (c.levels < 1 || c.levels > kMaxLevels) return fail(FHS_EINVAL, "levels must be in 1..6");
  if (c.precision != FHS_PRECISION_FP32 && c.precision != FHS_PRECISION_MIXED)
    return fail(FHS_EINVAL, "precision must be FHS_PRECISION_FP32 or FHS_PRECISION_MIXED");
  if (static_cast<int64_t>(c.ny) * c.nx * c.nchan > (int64_t(1) << 40)) return fail(FHS_EUNSUPPORTED, "cube too large");
  if (c.spectral_overlap < 0) return fail(FHS_EINVAL, "negative spectral overlap");
  if (c.spectral_overlap > 0) {
    if (c.n_sub < 2) return fail(FHS_EINVAL, "spectral overlap needs at least two sub-cubes");
    if (c.spectral_overlap > c.nchan / c.n_sub) return fail(FHS_EINVAL, "spectral overlap larger than a block");
    if (c.nchan / c.n_sub + c.spectral_overlap > kMaxLc)
      return fail(FHS_EUNSUPPORTED, "more than 64 channels per facet matrix");
    if (c.precision != FHS_PRECISION_FP32)
      return fail(FHS_EUNSUPPORTED, "spectral overlap is supported in the FP32 form only");
  }

  fhs_plan *p = new (std::nothrow) fhs_plan();
  if (!p) return fail(FHS_ENOMEM, "out of host memory");
  p->cfg = c;
  p->L = c.nchan;
  p->C = c.n_sub;
  p->Lc = c.nchan / c.n_sub;
  p->Q = c.qy * c.qx;
  // lanes per sub-cube: a power of two >= L_c, at least 4; L_c = 6, 10, 12,
  // 18 and 20 run dense (10, 6, 5, 3 and 3 segments per wave instead of 8, 4,
  // 4, 2 and 2 padded ones)
  int lcp = 4;
  while (lcp < p->Lc) lcp *= 2;
#ifndef FHS_DENSE_LANES
#define FHS_DENSE_LANES 1
#endif
  if (FHS_DENSE_LANES && (p->Lc == 6 || p->Lc == 10 || p->Lc == 12 || p->Lc == 18 || p->Lc == 20)) lcp = p->Lc;
  p->Lcp = lcp;
  p->so = c.spectral_overlap;
  p->Ln = p->Lc + p->so;
  p->lc16 = (p->Ln + 15) / 16 * 16;

  // tiles
  p->ty.resize(c.qy + 1);
  p->tx.resize(c.qx + 1);
  for (int s = 0; s <= c.qy; ++s) p->ty[s] = static_cast<int>(static_cast<int64_t>(s) * c.ny / c.qy);
  for (int s = 0; s <= c.qx; ++s) p->tx[s] = static_cast<int>(static_cast<int64_t>(s) * c.nx / c.qx);
  for (int s = 0; s < c.qy; ++s)
    if (c.qy > 1 && c.overlap_y > p->ty[s + 1] - p->ty[s]) {
      delete p;
      return fail(FHS_EINVAL, "overlap_y larger than a tile");
    }
  for (int s = 0; s < c.qx; ++s)
    if (c.qx > 1 && c.overlap_x > p->tx[s + 1] - p->tx[s]) {
      delete p;
      return fail(FHS_EINVAL, "overlap_x larger than a tile");
    }

  // facets, f = c * Q + sy * qx + sx
  int64_t poff = 0;
  p->max_rows = 0;
  for (int cc = 0; cc < p->C; ++cc)
    for (int sy = 0; sy < c.qy; ++sy)
      for (int sx = 0; sx < c.qx; ++sx) {
        fhs_plan::Facet f{};
        f.c = cc;
        f.sy = sy;
        f.sx = sx;
        f.ty0 = p->ty[sy];
        f.ty1 = p->ty[sy + 1];
        f.tx0 = p->tx[sx];
        f.tx1 = p->tx[sx + 1];
        f.wy0 = sy > 0 ? f.ty0 - c.overlap_y : f.ty0;
        f.wx0 = sx > 0 ? f.tx0 - c.overlap_x : f.tx0;
        f.wy1 = f.ty1;
        f.wx1 = f.tx1;
        f.rows = static_cast<int64_t>(f.wy1 - f.wy0) * (f.wx1 - f.wx0);
        f.poff = poff;
        poff += f.rows * p->Ln;
        if (f.rows > p->max_rows) p->max_rows = static_cast<int>(f.rows);
        p->facets.push_back(f);
      }
  p->n_p = poff;
  p->p_sub = poff / p->C;

  // wavelet bands in storage order
  int64_t off = 0;
  for (int b = 0; b < kBases; ++b) {
    const int taps = 2 * (b + 1);
    p->ntap[b] = taps;
    std::vector<long double> h;
    try {
      h = daubechies(b + 1);
    } catch (...) {
      delete p;
      return fail(FHS_EINVAL, "filter derivation failed");
    }
    for (int m = 0; m < kMaxTap; ++m) {
      p->h[b][m] = m < taps ? static_cast<float>(h[m]) : 0.0f;
      // g[m] = (-1)^m h[L-1-m]
      p->g[b][m] = m < taps ? static_cast<float>(((m & 1) ? -1.0L : 1.0L) * h[taps - 1 - m]) : 0.0f;
    }
    p->band_first[b] = static_cast<int64_t>(p->bands.size());
    int ny = c.ny, nx = c.nx;
    for (int j = 0; j < c.levels; ++j) {
      const int Ky = (ny + taps - 1) / 2, Kx = (nx + taps - 1) / 2;
      p->in_ny[b][j] = ny;
      p->in_nx[b][j] = nx;
      p->Ky[b][j] = Ky;
      p->Kx[b][j] = Kx;
      for (int s = 0; s < 3; ++s) {
        p->bands.push_back({Ky, Kx, off, j + 1});
        off += static_cast<int64_t>(Ky) * Kx;
      }
      // coefficients of this level owned by each facet (per axis): b_j(s) =
      // ceil((b_{j-1}(s) - 1) / 2) from the tile starts, the last facet
      // owning the tail (the faceted transform of Sec. 2.4.2)
      const std::vector<int> &py = j == 0 ? p->ty : p->own_y[b][j - 1];
      const std::vector<int> &px = j == 0 ? p->tx : p->own_x[b][j - 1];
      std::vector<int> oy(c.qy + 1), ox(c.qx + 1);
      oy[0] = ox[0] = 0;
      for (int sy = 1; sy < c.qy; ++sy) oy[sy] = py[sy] / 2;  // = ceil((b - 1) / 2), b >= 1
      for (int sx = 1; sx < c.qx; ++sx) ox[sx] = px[sx] / 2;
      oy[c.qy] = Ky;
      ox[c.qx] = Kx;
      p->own_y[b][j] = oy;
      p->own_x[b][j] = ox;
      ny = Ky;
      nx = Kx;
    }
    p->bands.push_back({ny, nx, off, c.levels});
    off += static_cast<int64_t>(ny) * nx;
  }
  p->bands.push_back({c.ny, c.nx, off, 0});
  off += static_cast<int64_t>(c.ny) * c.nx;
  p->I = off;
  // owner tables of the randomized step: facet row / column owning each
  // coefficient row / column of every basis and level, and each pixel row /
  // column of the Dirac band (its tile)
  {
    auto append = [&](const std::vector<int> &bounds, int n) {
      const int32_t at = static_cast<int32_t>(p->own_tab.size());
      for (int s = 0; s + 1 < static_cast<int>(bounds.size()); ++s)
        for (int i = bounds[s]; i < bounds[s + 1]; ++i) p->own_tab.push_back(static_cast<uint8_t>(s));
      if (static_cast<int32_t>(p->own_tab.size()) - at != n) return -1;
      return static_cast<int>(at);
    };
    bool okt = true;
    for (int b = 0; b < kBases; ++b)
      for (int j = 0; j < c.levels; ++j) {
        p->own_r[b][j] = append(p->own_y[b][j], p->Ky[b][j]);
        p->own_c[b][j] = append(p->own_x[b][j], p->Kx[b][j]);
        okt = okt && p->own_r[b][j] >= 0 && p->own_c[b][j] >= 0;
      }
    p->own_dr = append(p->ty, c.ny);
    p->own_dc = append(p->tx, c.nx);
    if (!okt || p->own_dr < 0 || p->own_dc < 0) {
      delete p;
      return fail(FHS_EINVAL, "internal: ownership does not cover the bands");
    }
  }
  if (static_cast<int64_t>(p->C) * p->I * 4 >= (int64_t{1} << 31)) {
    delete p;
    return fail(FHS_EUNSUPPORTED, "theta (C * I floats) must be smaller than 2 GiB");
  }

  // workspace: low-low bands of every basis and level but the last, then the
  // nuclear scratch (partial Gram matrices, K matrices, singular values)
  int64_t ws = 0;
  for (int b = 0; b < kBases; ++b)
    for (int j = 0; j < kMaxLevels; ++j) {
      p->ws_ll[b][j] = -1;
      if (j < c.levels - 1) {
        p->ws_ll[b][j] = ws;
        ws = align256(ws + static_cast<int64_t>(p->Ky[b][j]) * p->Kx[b][j] * p->L * 4);
      }
    }
  // nuclear kernels: segments of S pixels of one window row, chunks of whole
  // window rows of about 4096 pixels per workgroup
  for (const auto &f : p->facets) {
    p->max_hx = std::max(p->max_hx, f.wx1 - f.wx0);
    p->max_hy = std::max(p->max_hy, f.wy1 - f.wy0);
  }
  {
    fhs_tuning &t = p->tune;
    for (int j = 0; j < kMaxLevels; ++j) t.ana_rows[j] = 64;
    t.ana_phase = 4;
    t.syn_rows = 64;
    t.fin_rows = 128;
    t.fin_waves = 8;
    // largest S (at most 64 / 32 / 16 by channel count) whose reconstruction
    // tile fits in 64 KB of LDS
    t.nuc_seg = 64;
    while (t.nuc_seg > 16 && nuc_recon_lds(p, t.nuc_seg) > 65536) t.nuc_seg /= 2;
    t.nuc_chunk_rows = std::max(1, 4096 / p->max_hx);
    t.concurrent = 1;
    t.ana_direct = 0;
    t.ana_order = 0;
    p->nuc_chunk_min = std::max(1, t.nuc_chunk_rows / 2);
    p->gram_chunks = (p->max_hy + p->nuc_chunk_min - 1) / p->nuc_chunk_min;
  }
  const int64_t nf = static_cast<int64_t>(p->facets.size());
  p->ws_gram = ws;
  ws = align256(ws + nf * p->gram_chunks * p->lc16 * p->lc16 * 8);
  p->ws_kmat = ws;
  ws = align256(ws + nf * p->lc16 * p->lc16 * 8);
  p->ws_sig = ws;
  ws = align256(ws + nf * p->Ln * 8);
  // closure sums: about 2048 blocks of whole pixel groups
  {
    const int64_t npix = static_cast<int64_t>(c.ny) * c.nx;
    const int64_t G = std::max(1, 256 / p->L);
    const int64_t per = (npix + G * 2048 - 1) / (G * 2048);
    p->red_ppb = G * std::max<int64_t>(1, per);
    p->red_blocks = static_cast<int>((npix + p->red_ppb - 1) / p->red_ppb);
  }
  p->ws_red = ws;
  // (closure: one or two sums per channel and block; metrics: four)
  ws = align256(ws + static_cast<int64_t>(p->red_blocks) * std::max(4 * p->L, 2) * 8);
  p->ws_factor = ws;
  ws = align256(ws + static_cast<int64_t>(p->L) * 8);
  // per-channel sums read back by the reweighting solve
  p->ws_ctl = ws;
  ws = align256(ws + static_cast<int64_t>(p->L) * 2 * 8);
  // per-sub-cube activity flags of the reweighting solve
  p->ws_active = ws;
  ws = align256(ws + static_cast<int64_t>(p->C) * 4);
  // diagnostic counters (cleared when the workspace is attached)
  p->ws_diag = ws;
  ws = align256(ws + 2 * 4);
  // owner tables (copied when the workspace is attached)
  p->ws_own = ws;
  ws = align256(ws + static_cast<int64_t>(p->own_tab.size()));
  p->ws_bytes = ws;
  *out = p;
  return FHS_OK;
}

void fhs_plan_destroy(fhs_plan *plan) {
  if (!plan) return;
  if (!plan->prof_events.empty()) prof_release(plan);
  if (plan->side) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(plan->side));
    (void)hipStreamDestroy(static_cast<hipStream_t>(plan->side));
    (void)hipEventDestroy(static_cast<hipEvent_t>(plan->ev_fork));
    (void)hipEventDestroy(static_cast<hipEvent_t>(plan->ev_join));
  }
  delete plan;
}

int fhs_plan_sizes(const fhs_plan *p, fhs_sizes *out) {
  if (!p || !out) return fail(FHS_EINVAL, "fhs_plan_sizes: null argument");
  out->n_x = static_cast<int64_t>(p->cfg.ny) * p->cfg.nx * p->L;
  out->n_p = p->n_p;
  out->n_coef = p->I;
  out->n_w = p->I * p->L;
  out->n_theta = p->I * p->C;
  out->n_facets = static_cast<int64_t>(p->facets.size());
  out->n_theta_bar = out->n_facets * p->Ln;
  out->n_bands = static_cast<int64_t>(p->bands.size());
  out->workspace_bytes = p->ws_bytes;
  return FHS_OK;
}

int fhs_plan_facet(const fhs_plan *p, int32_t f, int64_t out[12]) {
  if (!p || !out) return fail(FHS_EINVAL, "fhs_plan_facet: null argument");
  if (f < 0 || f >= static_cast<int32_t>(p->facets.size())) return fail(FHS_EINVAL, "facet index out of range");
  const auto &F = p->facets[f];
  const int64_t v[12] = {F.c, F.sy, F.sx, F.ty0, F.ty1, F.tx0, F.tx1, F.wy0, F.wy1, F.wx0, F.wx1, F.poff};
  std::memcpy(out, v, sizeof(v));
  return FHS_OK;
}

int fhs_plan_band(const fhs_plan *p, int32_t k, int64_t out[4]) {
  if (!p || !out) return fail(FHS_EINVAL, "fhs_plan_band: null argument");
  if (k < 0 || k >= static_cast<int32_t>(p->bands.size())) return fail(FHS_EINVAL, "band index out of range");
  const auto &B = p->bands[k];
  out[0] = B.rows;
  out[1] = B.cols;
  out[2] = B.off;
  out[3] = B.level;
  return FHS_OK;
}

int fhs_plan_heuristics(const fhs_plan *p, const double *sigma_bar, double *mu, double *mu_bar) {
  if (!p || !sigma_bar || !mu || !mu_bar) return fail(FHS_EINVAL, "fhs_plan_heuristics: null argument");
  double m, s;
  chi_mean_std(static_cast<double>(p->Lc), &m, &s);
  for (int c = 0; c < p->C; ++c) {
    if (!(sigma_bar[c] > 0)) return fail(FHS_EINVAL, "sigma_bar must be positive");
    mu[c] = sigma_bar[c] * (m + s);
  }
  for (size_t f = 0; f < p->facets.size(); ++f) {
    // channels of the facet matrix: L_c, or with a spectral overlap the
    // block's plus the o before it (none before the first block)
    const int nc = p->so > 0 && p->facets[f].c > 0 ? p->Ln : p->Lc;
    const double n = static_cast<double>(p->facets[f].rows);
    const double J = std::min(n, static_cast<double>(nc));
    mu_bar[f] = sigma_bar[p->facets[f].c] * std::sqrt(n * nc / J);
  }
  return FHS_OK;
}

int fhs_plan_get_tuning(const fhs_plan *p, fhs_tuning *out) {
  if (!p || !out) return fail(FHS_EINVAL, "fhs_plan_get_tuning: null argument");
  *out = p->tune;
  return FHS_OK;
}

int fhs_plan_set_tuning(fhs_plan *p, const fhs_tuning *t) {
  if (!p || !t) return fail(FHS_EINVAL, "fhs_plan_set_tuning: null argument");
  for (int j = 0; j < kMaxLevels; ++j)
    if (t->ana_rows[j] < 8 || t->ana_rows[j] > 256 || t->ana_rows[j] % 8)
      return fail(FHS_EINVAL, "ana_rows must be multiples of 8 in 8..256");
  if (t->ana_phase != 1 && t->ana_phase != 2 && t->ana_phase != 4) return fail(FHS_EINVAL, "ana_phase must be 1, 2 or 4");
  if (t->syn_rows < 16 || t->syn_rows > 256 || t->syn_rows % 8)
    return fail(FHS_EINVAL, "syn_rows must be a multiple of 8 in 16..256");
  if (t->fin_rows < 16 || t->fin_rows > 512 || t->fin_rows % 8)
    return fail(FHS_EINVAL, "fin_rows must be a multiple of 8 in 16..512");
  if (t->nuc_seg != 16 && t->nuc_seg != 32 && t->nuc_seg != 64) return fail(FHS_EINVAL, "nuc_seg must be 16, 32 or 64");
  if (nuc_recon_lds(p, t->nuc_seg) > 160 * 1024) return fail(FHS_EINVAL, "nuc_seg: reconstruction tile exceeds the LDS");
  if (t->nuc_chunk_rows < p->nuc_chunk_min)
    return fail(FHS_EINVAL, "nuc_chunk_rows below the workspace's minimum (" + std::to_string(p->nuc_chunk_min) + ")");
  if (t->concurrent != 0 && t->concurrent != 1) return fail(FHS_EINVAL, "concurrent must be 0 or 1");
  if (t->ana_direct < 0 || t->ana_direct >= (1 << kMaxLevels))
    return fail(FHS_EINVAL, "ana_direct must be a bit mask of levels (0 .. 63)");
  if (t->fin_waves != 4 && t->fin_waves != 6 && t->fin_waves != 8) return fail(FHS_EINVAL, "fin_waves must be 4, 6 or 8");
  if (t->ana_order < 0 || t->ana_order >= (1 << kMaxLevels))
    return fail(FHS_EINVAL, "ana_order must be a bit mask of levels (0 .. 63)");
  p->tune = *t;
  return FHS_OK;
}

int fhs_plan_set_workspace(fhs_plan *p, void *dev_ptr, int64_t bytes) {
  if (!p) return fail(FHS_EINVAL, "fhs_plan_set_workspace: null plan");
  if (!dev_ptr || bytes < p->ws_bytes)
    return fail(FHS_EINVAL, "workspace missing or smaller than fhs_sizes.workspace_bytes");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return fail(FHS_EINVAL, "workspace must be 256-byte aligned");
  p->ws = dev_ptr;
  p->ws_given = bytes;
  if (hipMemset(static_cast<char *>(dev_ptr) + p->ws_diag, 0, 2 * sizeof(unsigned)) != hipSuccess ||
      hipMemcpy(static_cast<char *>(dev_ptr) + p->ws_own, p->own_tab.data(), p->own_tab.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return fail(FHS_EHIP, "fhs_plan_set_workspace: initialising the workspace failed");
  if (!p->side) {
    // side stream (default priority) and fork / join events for the
    // concurrent nuclear chain; without them the step runs on one stream
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&a, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&b, hipEventDisableTiming) == hipSuccess) {
      p->side = s;
      p->ev_fork = a;
      p->ev_join = b;
    } else {
      if (s) (void)hipStreamDestroy(s);
      if (a) (void)hipEventDestroy(a);
      (void)hipGetLastError();
    }
  }
  return FHS_OK;
}

}  // extern "C"
