// Compute entry points of libfhs: argument checks and launch sequences.
// No device allocation, no host synchronisation: every call only enqueues
// kernels on the caller's stream, so a sequence of calls can be captured in a
// HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "fhs_internal.h"

using namespace fhs;

namespace {

constexpr int kMaxDiracWg = 8192;
#ifndef FHS_ANA_LDS_KB
#define FHS_ANA_LDS_KB 80
#endif
constexpr int kAnaLdsBytes = FHS_ANA_LDS_KB * 1024;  // LDS budget of an analysis workgroup (two per CU)
constexpr int kAnaThreads = FHS_ANA_THREADS;          // upper bound on analysis workgroup size
constexpr int kCUs = 256;                              // compute units of an MI355X

int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

float *ws_f(const fhs_plan *p, int64_t off) { return reinterpret_cast<float *>(static_cast<char *>(ws_base(p)) + off); }
double *ws_d(const fhs_plan *p, int64_t off) {
  return reinterpret_cast<double *>(static_cast<char *>(ws_base(p)) + off);
}

bool dense_width_h(int lcp) { return (lcp & (lcp - 1)) != 0; }
bool dense_lanes(const fhs_plan *p) { return dense_width_h(p->Lcp); }
int pow2_lanes(const fhs_plan *p) {  // the padded segment width of the plan's L_c
  int lcp = 4;
  while (lcp < p->Lc) lcp *= 2;
  return lcp;
}

// Coefficient columns per workgroup (each C segments of lcp lanes) and the
// workgroup size.  Dense widths: 64 / lcp whole segments per wave.
int thread_cfg_w(int lcp, int C, int *tkx1, int *nthreads, int max_threads) {
  if (dense_width_h(lcp)) {
    const int g = 64 / lcp, segs = (max_threads / 64) * g;
    if (segs < C) return fail(FHS_EUNSUPPORTED, "sub-cubes exceed the lane segments of a workgroup");
    *tkx1 = segs / C;
    *nthreads = (*tkx1 * C + g - 1) / g * 64;
    return FHS_OK;
  }
  const int per = lcp * C;
  if (per > 256) return fail(FHS_EUNSUPPORTED, "sub-cubes x padded channels per sub-cube exceed 256");
  *tkx1 = std::max(1, max_threads / per);
  *nthreads = *tkx1 * per;
  return FHS_OK;
}

int thread_cfg(const fhs_plan *p, int *tkx1, int *nthreads, int max_threads = 256) {
  return thread_cfg_w(p->Lcp, p->C, tkx1, nthreads, max_threads);
}

int check_plan(const fhs_plan *p) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  return FHS_OK;
}

int64_t coef_off(const fhs_plan *p, int b, int j, int s) {  // s: 0 lh, 1 hl, 2 hh
  return p->bands[p->band_first[b] + 3 * j + s].off;
}
int64_t ll_off(const fhs_plan *p, int b) { return p->bands[p->band_first[b] + 3 * p->cfg.levels].off; }
int64_t dirac_off(const fhs_plan *p) { return p->bands.back().off; }

// LDS words of one phase buffer of the analysis for P steps: 2P staged rows,
// and for the dual update 4P W row runs and 4P theta segments.
int ana_lds_buf(const AnaArgs &a, int P) {
  int words = 2 * P * a.lds_row;
  if (a.mode == 1 || a.mode == 3) words += 4 * P * (kAnaLaneSeg + kAnaThSeg);
  return words;
}

int run_analysis(const fhs_plan *p, const float *x, float *w, float *theta, const double *mu, double inv_kappa,
                 int mode, void *stream, int fy = -1, int fx = -1, int level = -1, bool with_dirac = true,
                 const int32_t *active = nullptr, const uint8_t *sel = nullptr) {
  int tkx1, nth;
  if (int rc = thread_cfg(p, &tkx1, &nth, kAnaThreads)) return rc;
  const int TKX = tkx1;
  const int levels = p->cfg.levels;
  const bool facet = fy >= 0;
  for (int j = 0; j < levels; ++j) {
    if (level >= 0 && j != level) continue;
    AnaArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = w;
    a.theta = theta;
    a.mu = mu;
    a.inv_kappa = inv_kappa;
    a.I = p->I;
    a.theta_bytes = static_cast<int64_t>(p->C) * p->I * 4;
    a.L = p->L;
    a.C = p->C;
    a.Lc = p->Lc;
    a.Lcp = p->Lcp;
    a.tkx1 = tkx1;
    a.tky = p->tune.ana_rows[j];
    a.direct = (p->tune.ana_direct >> j) & 1;
    a.tile_major = (p->tune.ana_order >> j) & 1;
    a.f32 = ((mode == 1 || mode == 3) && p->cfg.precision == FHS_PRECISION_MIXED) ? 1 : 0;
    a.mode = mode;
    a.active = active;
    a.sel = sel;
    a.own = static_cast<const uint8_t *>(ws_base(p)) + p->ws_own;
    a.qy = p->cfg.qy;
    a.qx = p->cfg.qx;
    // staged row: [sub-cube][column][lane slot], columns of the widest filter
    // (plus one pad column per sub-cube block when there are several), in
    // whole copy chunks (256 words with 16-byte copies, else 64)
    a.vec4 = (p->L % 4 == 0 && p->Lc % 4 == 0) ? 1 : 0;
    // (the kernel copies 4 bytes per lane from the natural-order cube when
    // there are several sub-cubes: a sub-cube's channels are not contiguous)
    const bool v4 = a.vec4 && (p->C == 1 || j > 0 || p->so > 0);
    const int cw = v4 ? 256 : 64;
    const int ncp = 2 * TKX + kMaxTap - 2 + (p->C > 1 ? 1 : 0);
    const int nchunk = ceil_div(static_cast<int64_t>(p->C) * ncp * p->Lcp, cw);
    a.lds_row = nchunk * cw;
    if (nth < 64) return fail(FHS_EUNSUPPORTED, "analysis: fewer than 64 threads per workgroup");
    if (p->C * TKX > kAnaThSeg) return fail(FHS_EUNSUPPORTED, "analysis: more than 128 sub-cube columns per tile");
    const int tab_words = nchunk * 64;
    int tmax = 0;
    for (int b = 0; b < kBases; ++b) {
      AnaBand &B = a.b[b];
      B.in = j == 0 ? x : ws_f(p, p->ws_ll[b][j - 1]);
      // (contiguous sub-cubes: the cube's channel order is the positions order)
      B.in_natural = j == 0 && p->so == 0 ? 1 : 0;
      B.in_ny = p->in_ny[b][j];
      B.in_nx = p->in_nx[b][j];
      B.ll_out = j < levels - 1 ? ws_f(p, p->ws_ll[b][j]) : nullptr;
      B.Ky = p->Ky[b][j];
      B.Kx = p->Kx[b][j];
      B.ky_begin = facet ? p->own_y[b][j][fy] : 0;
      B.ky_end = facet ? p->own_y[b][j][fy + 1] : B.Ky;
      B.kx_begin = facet ? p->own_x[b][j][fx] : 0;
      B.kx_end = facet ? p->own_x[b][j][fx + 1] : B.Kx;
      B.strips = std::max(0, ceil_div(B.kx_end - B.kx_begin, TKX));
      B.yblocks = std::max(0, ceil_div(B.ky_end - B.ky_begin, a.tky));
      B.ntap = p->ntap[b];
      B.own_r = p->own_r[b][j];
      B.own_c = p->own_c[b][j];
      for (int s = 0; s < 3; ++s) B.off[s] = coef_off(p, b, j, s);
      B.off[3] = j == levels - 1 ? ll_off(p, b) : -1;
      tmax = std::max(tmax, B.strips * B.yblocks);
    }
    a.tiles_per_xcd = ceil_div(tmax, 8);
    a.nbase_wg = 64 * a.tiles_per_xcd;
    // steps per phase: the most up to the tuned value whose double buffer fits
    // the LDS budget; a launch with no more workgroups than two per CU (the
    // deeper levels) may take the whole LDS of a CU per workgroup
    const int budget = a.nbase_wg <= 2 * kCUs ? 160 * 1024 : kAnaLdsBytes;
    a.P = 1;
    for (int P = p->tune.ana_phase; P >= 1; P /= 2)
      if ((2 * ana_lds_buf(a, P) + tab_words) * 4 <= budget || P == 1) {
        a.P = P;
        break;
      }
    a.lds_buf = ana_lds_buf(a, a.P);
    a.lds_wv = 2 * a.P * a.lds_row;
    a.lds_th = a.lds_wv + 4 * a.P * kAnaLaneSeg;
    a.lds_tab = 2 * a.lds_buf;
    a.lds_words = a.lds_tab + tab_words;
    if (a.lds_words * 4 > 160 * 1024) return fail(FHS_EUNSUPPORTED, "analysis: LDS tile exceeds 160 KB");
    if (j == 0) {
      AnaBand &D = a.b[kBases];
      D.in = x;
      D.in_natural = p->so == 0 ? 1 : 0;
      D.in_ny = p->cfg.ny;
      D.in_nx = p->cfg.nx;
      D.off[0] = dirac_off(p);
      D.own_r = p->own_dr;
      D.own_c = p->own_dc;
      D.ky_begin = facet ? p->ty[fy] : 0;
      D.ky_end = facet ? p->ty[fy + 1] : p->cfg.ny;
      D.kx_begin = facet ? p->tx[fx] : 0;
      D.kx_end = facet ? p->tx[fx + 1] : p->cfg.nx;
      // grid-stride workgroups of the Dirac-band kernel (kDiracE pixels in flight per thread)
      const int64_t npix = static_cast<int64_t>(D.ky_end - D.ky_begin) * (D.kx_end - D.kx_begin);
      const int ppw = kDiracThreads / (p->C * pow2_lanes(p));  // (padded segments)
      if (ppw < 1) return fail(FHS_EUNSUPPORTED, "Dirac band: sub-cubes exceed the lane segments of a workgroup");
      D.strips = npix > 0 && with_dirac
                     ? std::max(1, std::min(kMaxDiracWg, ceil_div(npix, static_cast<int64_t>(kDiracE) * ppw)))
                     : 0;
    }
    const int kid = j == 0 ? FHS_K_ANALYSIS_L1 : FHS_K_ANALYSIS;
    prof_begin(p, kid, stream);
    const int rc = launch_analysis(a, nth, j == 0, stream);
    prof_end(p, kid, stream);
    if (rc) return rc;
  }
  return FHS_OK;
}

// coefficient columns (strips of tk) covering output samples [b, e)
int syn_strips(int b, int e, int tk) { return e > b ? ceil_div((e - 1) / 2 - b / 2 + 1, tk) : 0; }

// x = beta x + alpha Psi w.  Facet (fy, fx) >= 0 restricts the outputs to the
// samples that facet owns, level >= 0 to one level (0 = the final level-1
// pass): the per-facet execution form.
// xin non-null: the level-1 pass also performs the Dirac band's l21 dual
// update (left out of the analysis) with input xin, weights theta, mu, 1/kappa.
int run_synthesis(const fhs_plan *p, const float *w, float *x, float alpha, float beta, void *stream, int fy = -1,
                  int fx = -1, int level = -1, const float *xin = nullptr, const float *theta = nullptr,
                  const double *mu = nullptr, double inv_kappa = 0.0, const int32_t *active = nullptr) {
  int tk, nth;
  if (int rc = thread_cfg(p, &tk, &nth, FHS_SYN_THREADS)) return rc;
  const int L = p->L, levels = p->cfg.levels;
  const bool facet = fy >= 0;
  for (int j = levels - 1; j >= 1; --j) {  // 0-based level j -> writes low-low band of level j-1
    if (level >= 0 && j != level) continue;
    SynArgs s;
    std::memset(&s, 0, sizeof(s));
    s.L = L;
    s.Lcp = p->Lcp;
    s.C = p->C;
    s.Lc = p->Lc;
    s.tk = tk;
    s.ty = p->tune.syn_rows;
    int prefix = 0;
    for (int b = 0; b < kBases; ++b) {
      SynBand &B = s.b[b];
      B.ll = j == levels - 1 ? w + ll_off(p, b) * L : ws_f(p, p->ws_ll[b][j]);
      B.lh = w + coef_off(p, b, j, 0) * L;
      B.hl = w + coef_off(p, b, j, 1) * L;
      B.hh = w + coef_off(p, b, j, 2) * L;
      B.out = ws_f(p, p->ws_ll[b][j - 1]);
      B.Ky = p->Ky[b][j];
      B.Kx = p->Kx[b][j];
      B.ny = p->in_ny[b][j];
      B.nx = p->in_nx[b][j];
      B.y_begin = facet ? p->own_y[b][j - 1][fy] : 0;
      B.y_end = facet ? p->own_y[b][j - 1][fy + 1] : B.ny;
      B.x_begin = facet ? p->own_x[b][j - 1][fx] : 0;
      B.x_end = facet ? p->own_x[b][j - 1][fx + 1] : B.nx;
      B.strips = syn_strips(B.x_begin, B.x_end, tk);
      B.yblocks = std::max(0, ceil_div(B.y_end - B.y_begin, s.ty));
      B.ntap = p->ntap[b];
      s.wg_prefix[b] = prefix;
      prefix += B.strips * B.yblocks;
    }
    s.wg_prefix[kBases] = prefix;
    if (prefix == 0) continue;
    prof_begin(p, FHS_K_SYNTHESIS, stream);
    const int rc = launch_synthesis(s, nth, stream);
    prof_end(p, FHS_K_SYNTHESIS, stream);
    if (rc) return rc;
  }
  if (level > 0) return FHS_OK;
  // level 1: its own workgroup size (fin_waves) and padded lane segments
  // (measured faster there than the dense ones)
  const int lcp_fin = pow2_lanes(p);
  if (int rc = thread_cfg_w(lcp_fin, p->C, &tk, &nth, 64 * p->tune.fin_waves)) return rc;
  SynFinalArgs f;
  std::memset(&f, 0, sizeof(f));
  for (int b = 0; b < kBases; ++b) {
    SynBand &B = f.b[b];
    B.ll = levels == 1 ? w + ll_off(p, b) * L : ws_f(p, p->ws_ll[b][0]);
    B.lh = w + coef_off(p, b, 0, 0) * L;
    B.hl = w + coef_off(p, b, 0, 1) * L;
    B.hh = w + coef_off(p, b, 0, 2) * L;
    B.Ky = p->Ky[b][0];
    B.Kx = p->Kx[b][0];
    B.ny = p->cfg.ny;
    B.nx = p->cfg.nx;
    B.ntap = p->ntap[b];
  }
  f.dirac = const_cast<float *>(w) + dirac_off(p) * L;
  f.x = x;
  f.xin = xin;
  f.active = active;
  f.theta = theta;
  f.mu = mu;
  f.inv_kappa = inv_kappa;
  f.I = p->I;
  f.dirac_row = dirac_off(p);
  f.theta_bytes = static_cast<int64_t>(p->C) * p->I * 4;
  f.alpha = alpha;
  f.beta = beta;
  f.contig = p->so > 0 ? 1 : 0;
  f.ny = p->cfg.ny;
  f.nx = p->cfg.nx;
  f.L = L;
  f.Lcp = lcp_fin;
  f.C = p->C;
  f.Lc = p->Lc;
  f.tk = tk;
  f.ty = p->tune.fin_rows;
  f.y_begin = facet ? p->ty[fy] : 0;
  f.y_end = facet ? p->ty[fy + 1] : p->cfg.ny;
  f.x_begin = facet ? p->tx[fx] : 0;
  f.x_end = facet ? p->tx[fx + 1] : p->cfg.nx;
  f.strips = syn_strips(f.x_begin, f.x_end, tk);
  f.yblocks = ceil_div(f.y_end - f.y_begin, f.ty);
  // group 0 (timed as SYNTH_FINAL_A), groups 1 and 2 (timed together as SYNTH_FINAL_B)
  for (int grp = 0; grp < 3; ++grp) {
    const int kid = grp == 0 ? FHS_K_SYNTH_FINAL_A : FHS_K_SYNTH_FINAL_B;
    if (grp != 2) prof_begin(p, kid, stream);
    const int rc = launch_synthesis_final(f, nth, grp, stream);
    if (grp != 1) prof_end(p, kid, stream);
    if (rc) return rc;
  }
  return FHS_OK;
}

void fill_geom(const fhs_plan *p, NucGeom &g) {
  std::memset(&g, 0, sizeof(g));
  g.ny = p->cfg.ny;
  g.nx = p->cfg.nx;
  g.L = p->L;
  g.C = p->C;
  g.Lc = p->Ln;
  g.spec = p->so > 0 ? 1 : 0;
  g.sb = p->Lc;
  g.so = p->so;
  g.qy = p->cfg.qy;
  g.qx = p->cfg.qx;
  g.oy = p->cfg.overlap_y;
  g.ox = p->cfg.overlap_x;
  for (int s = 0; s <= g.qy; ++s) g.ty[s] = p->ty[s];
  for (int s = 0; s <= g.qx; ++s) g.tx[s] = p->tx[s];
  g.py[0] = 0;
  for (int s = 0; s < g.qy; ++s) {
    const int w0 = s > 0 ? p->ty[s] - g.oy : p->ty[s];
    g.py[s + 1] = g.py[s] + (p->ty[s + 1] - w0);
  }
  g.px[0] = 0;
  for (int s = 0; s < g.qx; ++s) {
    const int w0 = s > 0 ? p->tx[s] - g.ox : p->tx[s];
    g.px[s + 1] = g.px[s] + (p->tx[s + 1] - w0);
  }
  g.p_sub = p->p_sub;
}

int run_gather(const fhs_plan *p, const float *pdual, float *grad, double zeta, float beta, void *stream,
               int fy = -1, int fx = -1);

// mode 0: dual update of p (+ gather unless no_gather); mode 1: weights only
// q >= 0: only spatial facet q (all its sub-cubes), without the gather: the
// per-facet execution form.
int run_nuclear(const fhs_plan *p, const float *x, float *pdual, const double *theta_bar, const double *mu_bar,
                double zeta, double *theta_bar_out, float *grad, float beta, int mode, void *stream,
                bool no_gather = false, int q = -1, const int32_t *active = nullptr,
                const uint8_t *sel = nullptr) {
  NucArgs a;
  std::memset(&a, 0, sizeof(a));
  fill_geom(p, a.g);
  a.x = x;
  a.p = pdual;
  a.gram = ws_d(p, p->ws_gram);
  a.kmat = ws_d(p, p->ws_kmat);
  a.sig = ws_d(p, p->ws_sig);
  a.theta_bar = theta_bar;
  a.mu_bar = mu_bar;
  a.theta_bar_out = theta_bar_out;
  a.inv_zeta = 1.0 / zeta;
  a.chunk_wrows = p->tune.nuc_chunk_rows;
  a.chunks = ceil_div(p->max_hy, a.chunk_wrows);  // <= p->gram_chunks (the workspace's slots)
  a.seg = p->tune.nuc_seg;
  a.lc16 = p->lc16;
  a.mode = mode;
  a.diag = reinterpret_cast<unsigned *>(static_cast<char *>(ws_base(p)) + p->ws_diag);
  a.bf16 = (mode == 0 && p->cfg.precision == FHS_PRECISION_MIXED) ? 1 : 0;
  a.q0 = q >= 0 ? q : 0;
  a.eig_q = q;
  a.active = active;
  a.sel = mode == 0 ? sel : nullptr;
  const int nspatial = q >= 0 ? 1 : p->Q;
  const int nf = q >= 0 ? p->C : static_cast<int>(p->facets.size());
  int rc;
  prof_begin(p, FHS_K_NUC_GRAM, stream);
  rc = launch_nuc_gram(a, nspatial, stream);
  prof_end(p, FHS_K_NUC_GRAM, stream);
  if (rc) return rc;
  prof_begin(p, FHS_K_NUC_EIG, stream);
  rc = launch_nuc_eig(a, nf, stream);
  prof_end(p, FHS_K_NUC_EIG, stream);
  if (rc) return rc;
  if (mode == 1) return FHS_OK;
  prof_begin(p, FHS_K_NUC_RECON, stream);
  rc = launch_nuc_recon(a, nspatial, stream);
  prof_end(p, FHS_K_NUC_RECON, stream);
  if (rc) return rc;
  if (no_gather || q >= 0) return FHS_OK;
  return run_gather(p, pdual, grad, zeta, beta, stream);
}

// fy >= 0: only the tile of facet (fy, fx).
int run_gather(const fhs_plan *p, const float *pdual, float *grad, double zeta, float beta, void *stream, int fy,
               int fx) {
  GatherArgs ga;
  std::memset(&ga, 0, sizeof(ga));
  fill_geom(p, ga.g);
  ga.y_begin = fy >= 0 ? p->ty[fy] : 0;
  ga.y_end = fy >= 0 ? p->ty[fy + 1] : p->cfg.ny;
  ga.x_begin = fy >= 0 ? p->tx[fx] : 0;
  ga.x_end = fy >= 0 ? p->tx[fx + 1] : p->cfg.nx;
  ga.p = pdual;
  ga.grad = grad;
  ga.zeta = zeta;
  ga.beta = beta;
  prof_begin(p, FHS_K_NUC_GATHER, stream);
  const int rc = launch_nuc_gather(ga, stream);
  prof_end(p, FHS_K_NUC_GATHER, stream);
  return rc;
}

int l21_update(const fhs_plan *p, const float *xcheck, float *w, const float *theta, const double *mu, double kappa,
               float *grad, float beta, void *stream, const int32_t *active) {
  // (the Dirac band's dual update runs inside the level-1 synthesis, which
  // reads the updated coefficient right away)
  if (int rc = run_analysis(p, xcheck, w, const_cast<float *>(theta), mu, 1.0 / kappa, 1, stream, -1, -1, -1, false,
                            active))
    return rc;
  return run_synthesis(p, w, grad, static_cast<float>(kappa), beta, stream, -1, -1, -1, xcheck, theta, mu, 1.0 / kappa,
                       active);
}

// The l21 dual update of the rows owned by the selected facets (randomized
// step): the Dirac band is updated by the analysis (masked by tile), and the
// synthesis reads every row as it stands.
int l21_update_select(const fhs_plan *p, const float *xcheck, float *w, const float *theta, const double *mu,
                      double kappa, float *grad, float beta, void *stream, const uint8_t *sel) {
  if (int rc = run_analysis(p, xcheck, w, const_cast<float *>(theta), mu, 1.0 / kappa, 3, stream, -1, -1, -1, true,
                            nullptr, sel))
    return rc;
  return run_synthesis(p, w, grad, static_cast<float>(kappa), beta, stream);
}

int l21_step(const fhs_plan *p, const float *xcheck, float *w, const float *theta, const double *mu, double kappa,
             float *grad, void *stream, const int32_t *active, const uint8_t *sel) {
  return sel ? l21_update_select(p, xcheck, w, theta, mu, kappa, grad, 0.0f, stream, sel)
             : l21_update(p, xcheck, w, theta, mu, kappa, grad, 0.0f, stream, active);
}

}  // namespace

namespace fhs {

int facet_prox_step(const fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                    const double *theta_bar, const double *mu, const double *mu_bar, double zeta, double kappa,
                    float *grad, void *stream, const int32_t *active, const uint8_t *sel) {
  if (!p->side || !p->tune.concurrent) {
    if (int rc = l21_step(p, xcheck, w, theta, mu, kappa, grad, stream, active, sel)) return rc;
    return run_nuclear(p, xcheck, pdual, theta_bar, mu_bar, zeta, nullptr, grad, 1.0f, 0, stream, false, -1, active,
                       sel);
  }
  // The two dual updates are independent until the gather: the nuclear
  // chain (Gram, eigendecomposition, reconstruction) runs on the plan's side
  // stream beside the wavelet chain, and the gather waits for both.
  hipStream_t s0 = static_cast<hipStream_t>(stream), s1 = static_cast<hipStream_t>(p->side);
  hipEvent_t fork = static_cast<hipEvent_t>(p->ev_fork), join = static_cast<hipEvent_t>(p->ev_join);
  if (hipEventRecord(fork, s0) != hipSuccess || hipStreamWaitEvent(s1, fork, 0) != hipSuccess)
    return fail(FHS_EHIP, "fork to the side stream failed");
  int rc = run_nuclear(p, xcheck, pdual, theta_bar, mu_bar, zeta, nullptr, grad, 1.0f, 0, s1, true, -1, active, sel);
  const bool joined = hipEventRecord(join, s1) == hipSuccess;
  if (rc == FHS_OK) rc = l21_step(p, xcheck, w, theta, mu, kappa, grad, stream, active, sel);
  if (!joined || hipStreamWaitEvent(s0, join, 0) != hipSuccess)
    return rc ? rc : fail(FHS_EHIP, "join of the side stream failed");
  if (rc) return rc;
  return run_gather(p, pdual, grad, zeta, 1.0f, stream);
}

int reweight(const fhs_plan *p, const float *x, const double *upsilon, const double *upsilon_bar, float *theta,
             double *theta_bar, void *stream, const int32_t *active) {
  if (int rc = run_nuclear(p, x, nullptr, nullptr, upsilon_bar, 1.0, theta_bar, nullptr, 0.0f, 1, stream, false, -1,
                           active))
    return rc;
  return run_analysis(p, x, nullptr, theta, upsilon, 1.0, 2, stream, -1, -1, -1, true, active);
}

}  // namespace fhs

extern "C" {

int fhs_sara_analysis(const fhs_plan *p, const float *x, float *w, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!x || !w) return fail(FHS_EINVAL, "fhs_sara_analysis: null array");
  return run_analysis(p, x, w, nullptr, nullptr, 1.0, 0, stream);
}

int fhs_sara_synthesis(const fhs_plan *p, const float *w, float *x, float alpha, float beta, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!x || !w) return fail(FHS_EINVAL, "fhs_sara_synthesis: null array");
  return run_synthesis(p, w, x, alpha, beta, stream);
}

int fhs_l21_dual_update(const fhs_plan *p, const float *xcheck, float *w, const float *theta, const double *mu,
                        double kappa, float *grad, float beta, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!xcheck || !w || !theta || !mu || !grad) return fail(FHS_EINVAL, "fhs_l21_dual_update: null array");
  if (!(kappa > 0)) return fail(FHS_EINVAL, "kappa must be positive");
  return l21_update(p, xcheck, w, theta, mu, kappa, grad, beta, stream, nullptr);
}

int fhs_nuclear_dual_update(const fhs_plan *p, const float *xcheck, float *pdual, const double *theta_bar,
                            const double *mu_bar, double zeta, float *grad, float beta, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!xcheck || !pdual || !theta_bar || !mu_bar || !grad) return fail(FHS_EINVAL, "fhs_nuclear_dual_update: null array");
  if (!(zeta > 0)) return fail(FHS_EINVAL, "zeta must be positive");
  return run_nuclear(p, xcheck, pdual, theta_bar, mu_bar, zeta, nullptr, grad, beta, 0, stream);
}

int fhs_facet_prox_step(const fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                        const double *theta_bar, const double *mu, const double *mu_bar, double zeta, double kappa,
                        float *grad, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!xcheck || !pdual || !w || !theta || !theta_bar || !mu || !mu_bar || !grad)
    return fail(FHS_EINVAL, "fhs_facet_prox_step: null array");
  if (!(zeta > 0) || !(kappa > 0)) return fail(FHS_EINVAL, "zeta and kappa must be positive");
  return facet_prox_step(p, xcheck, pdual, w, theta, theta_bar, mu, mu_bar, zeta, kappa, grad, stream, nullptr);
}

int fhs_facet_prox_step_select(const fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                               const double *theta_bar, const double *mu, const double *mu_bar, double zeta,
                               double kappa, const uint8_t *select, float *grad, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!xcheck || !pdual || !w || !theta || !theta_bar || !mu || !mu_bar || !select || !grad)
    return fail(FHS_EINVAL, "fhs_facet_prox_step_select: null array");
  if (!(zeta > 0) || !(kappa > 0)) return fail(FHS_EINVAL, "zeta and kappa must be positive");
  return facet_prox_step(p, xcheck, pdual, w, theta, theta_bar, mu, mu_bar, zeta, kappa, grad, stream, nullptr,
                         select);
}

int fhs_facet_prox_step_plain(const fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                              const double *theta_bar, const double *mu, const double *mu_bar, double zeta,
                              double kappa, float *grad, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!xcheck || !pdual || !w || !theta || !theta_bar || !mu || !mu_bar || !grad)
    return fail(FHS_EINVAL, "fhs_facet_prox_step_plain: null array");
  if (!(zeta > 0) || !(kappa > 0)) return fail(FHS_EINVAL, "zeta and kappa must be positive");
  const int qy = p->cfg.qy, qx = p->cfg.qx, levels = p->cfg.levels;
  // l21: analysis level by level, facet by facet in raster order (a facet's
  // window needs the low-low band its top / left neighbours own)
  for (int j = 0; j < levels; ++j)
    for (int sy = 0; sy < qy; ++sy)
      for (int sx = 0; sx < qx; ++sx)
        if (int rc = run_analysis(p, xcheck, w, const_cast<float *>(theta), mu, 1.0 / kappa, 1, stream, sy, sx, j))
          return rc;
  // synthesis coarse to fine, each facet writing the samples it owns
  for (int j = levels - 1; j >= 0; --j)
    for (int sy = 0; sy < qy; ++sy)
      for (int sx = 0; sx < qx; ++sx)
        if (int rc = run_synthesis(p, w, grad, static_cast<float>(kappa), 0.0f, stream, sy, sx, j)) return rc;
  // nuclear: facet by facet (all sub-cubes of a spatial facet together), then
  // the gather tile by tile
  for (int q = 0; q < p->Q; ++q)
    if (int rc = run_nuclear(p, xcheck, pdual, theta_bar, mu_bar, zeta, nullptr, grad, 1.0f, 0, stream, true, q))
      return rc;
  for (int sy = 0; sy < qy; ++sy)
    for (int sx = 0; sx < qx; ++sx)
      if (int rc = run_gather(p, pdual, grad, zeta, 1.0f, stream, sy, sx)) return rc;
  return FHS_OK;
}

int fhs_reweight(const fhs_plan *p, const float *x, const double *upsilon, const double *upsilon_bar, float *theta,
                 double *theta_bar, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!x || !upsilon || !upsilon_bar || !theta || !theta_bar) return fail(FHS_EINVAL, "fhs_reweight: null array");
  return reweight(p, x, upsilon, upsilon_bar, theta, theta_bar, stream, nullptr);
}

int fhs_plan_diagnostics(const fhs_plan *p, int64_t out[2], int32_t reset, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!out) return fail(FHS_EINVAL, "fhs_plan_diagnostics: null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned h[2] = {0, 0};
  void *d = static_cast<char *>(p->ws) + p->ws_diag;
  if (hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(FHS_EHIP, "fhs_plan_diagnostics: reading the counters failed");
  out[0] = h[0];
  out[1] = h[1];
  if (reset && (hipMemsetAsync(d, 0, sizeof(h), s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess))
    return fail(FHS_EHIP, "fhs_plan_diagnostics: clearing the counters failed");
  return FHS_OK;
}

}  // extern "C"
