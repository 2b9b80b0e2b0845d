// Whole PDFB iterations (Alg. 2) with the identity as measurement operator:
// the facet step, the data-fidelity dual, the primal update and the
// extrapolation, enqueued on one stream, and their capture into a HIP graph
// so that many iterations replay with one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <vector>

#include "fhs_internal.h"

using namespace fhs;

struct fhs_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t iterations = 0;
};

namespace {

int closure(const fhs_plan *p, float *x, float *xcheck, float *v, const float *y, const double *eps,
            const float *grad, double tau, double *xi, void *stream, const int32_t *active = nullptr) {
  ClosureArgs a{};
  a.x = x;
  a.xcheck = xcheck;
  a.v = v;
  a.y = y;
  a.grad = grad;
  a.eps = eps;
  a.part = reinterpret_cast<double *>(static_cast<char *>(p->ws) + p->ws_red);
  a.factor = reinterpret_cast<double *>(static_cast<char *>(p->ws) + p->ws_factor);
  a.xi = xi;
  a.active = active;
  a.tau = tau;
  a.npix = static_cast<int64_t>(p->cfg.ny) * p->cfg.nx;
  a.ppb = p->red_ppb;
  a.L = p->L;
  a.C = p->C;
  a.nblocks = p->red_blocks;
  a.contig = p->so > 0 ? 1 : 0;
  prof_begin(p, FHS_K_CLOSURE, stream);
  const int rc = launch_closure(a, stream);
  prof_end(p, FHS_K_CLOSURE, stream);
  return rc;
}

int check_state(const fhs_pdfb_state *s) {
  if (!s) return fail(FHS_EINVAL, "null PDFB state");
  if (!s->x || !s->xcheck || !s->p || !s->w || !s->v || !s->y || !s->eps || !s->theta || !s->theta_bar || !s->mu ||
      !s->mu_bar || !s->grad || !s->xi)
    return fail(FHS_EINVAL, "PDFB state: null array");
  if (!(s->tau > 0)) return fail(FHS_EINVAL, "tau must be positive");
  return FHS_OK;
}

// One PDFB iteration; xi[c] receives the relative variation of sub-cube c.
int iteration(const fhs_plan *p, const fhs_pdfb_state *s, double *xi, void *stream, const int32_t *active) {
  if (int rc = facet_prox_step(p, s->xcheck, s->p, s->w, s->theta, s->theta_bar, s->mu, s->mu_bar, s->zeta, s->kappa,
                               s->grad, stream, active))
    return rc;
  return closure(p, s->x, s->xcheck, s->v, s->y, s->eps, s->grad, s->tau, xi, stream, active);
}

// Per-channel sums of r^2 and (r - x)^2 into the workspace's control slot,
// then copied to host `out` [2L] (synchronizes `stream`).
int channel_sums(const fhs_plan *p, const float *r, const float *x, double *out, hipStream_t stream) {
  SnrArgs a{};
  a.ref = r;
  a.x = x;
  a.part = reinterpret_cast<double *>(static_cast<char *>(p->ws) + p->ws_red);
  a.sums = reinterpret_cast<double *>(static_cast<char *>(p->ws) + p->ws_ctl);
  a.npix = static_cast<int64_t>(p->cfg.ny) * p->cfg.nx;
  a.ppb = p->red_ppb;
  a.L = p->L;
  a.nblocks = p->red_blocks;
  if (int rc = launch_snr(a, stream)) return rc;
  if (hipMemcpyAsync(out, a.sums, sizeof(double) * 2 * p->L, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(FHS_EHIP, "reweighting solve: reading back channel sums failed");
  return FHS_OK;
}

}  // namespace

extern "C" {

int fhs_pdfb_closure(const fhs_plan *p, float *x, float *xcheck, float *v, const float *y, const double *eps,
                     const float *grad, double tau, double *xi, void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  if (!x || !xcheck || !v || !y || !eps || !grad || !xi) return fail(FHS_EINVAL, "fhs_pdfb_closure: null array");
  if (!(tau > 0)) return fail(FHS_EINVAL, "tau must be positive");
  return closure(p, x, xcheck, v, y, eps, grad, tau, xi, stream);
}

int fhs_snr(const fhs_plan *p, const float *x_ref, const float *x, const double *eps, double *snr, double *snr_log,
            void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  if (!x_ref || !x || !snr) return fail(FHS_EINVAL, "fhs_snr: null array");
  if (eps && !snr_log) return fail(FHS_EINVAL, "fhs_snr: snr_log is required with eps");
  SnrArgs a{};
  a.ref = x_ref;
  a.x = x;
  a.eps = eps;
  a.part = reinterpret_cast<double *>(static_cast<char *>(p->ws) + p->ws_red);
  a.snr = snr;
  a.snr_log = snr_log;
  a.npix = static_cast<int64_t>(p->cfg.ny) * p->cfg.nx;
  a.ppb = p->red_ppb;
  a.L = p->L;
  a.nblocks = p->red_blocks;
  return launch_snr(a, stream);
}

int fhs_pdfb_iteration(const fhs_plan *p, const fhs_pdfb_state *s, int32_t iter, void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  if (int rc = check_state(s)) return rc;
  if (iter < 0) return fail(FHS_EINVAL, "iteration index must be >= 0");
  if (!(s->zeta > 0) || !(s->kappa > 0)) return fail(FHS_EINVAL, "zeta and kappa must be positive");
  return iteration(p, s, s->xi + static_cast<int64_t>(iter) * p->C, stream, nullptr);
}

int fhs_reweighting_solve(const fhs_plan *p, const fhs_pdfb_state *s, const double *upsilon,
                          const double *upsilon_bar, float *x_prev, const fhs_solve_params *prm, int32_t *iters,
                          double *rw_xi, fhs_solve_report *report, void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  if (int rc = check_state(s)) return rc;
  if (!upsilon || !upsilon_bar || !x_prev || !prm) return fail(FHS_EINVAL, "fhs_reweighting_solve: null argument");
  if (p->so > 0)
    return fail(FHS_EUNSUPPORTED, "reweighting solve: overlapping spectral facets couple the sub-problems");
  if (prm->max_reweights < 0 || prm->min_iter < 0 || prm->max_iter < 1 || prm->max_iter < prm->min_iter)
    return fail(FHS_EINVAL, "reweighting solve: need max_reweights >= 0 and 1 <= max_iter, min_iter <= max_iter");
  if (!(prm->rw_tol >= 0) || !(prm->pdfb_tol >= 0) || !(prm->res_factor > 0))
    return fail(FHS_EINVAL, "reweighting solve: tolerances must be >= 0 and res_factor > 0");
  if (!(s->zeta > 0) || !(s->kappa > 0)) return fail(FHS_EINVAL, "zeta and kappa must be positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int L = p->L, C = p->C;
  const size_t cube_bytes = static_cast<size_t>(p->cfg.ny) * p->cfg.nx * L * sizeof(float);
  constexpr double kInf = std::numeric_limits<double>::infinity();
  std::vector<double> h(2 * static_cast<size_t>(L));
  // ||eps_c|| over the channels c, c + C, ... of each sub-cube
  if (hipMemcpyAsync(h.data(), s->eps, sizeof(double) * L, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(FHS_EHIP, "reweighting solve: reading eps failed");
  std::vector<double> res_bound(C, 0.0);
  for (int l = 0; l < L; ++l) res_bound[l % C] += h[l] * h[l];
  for (int c = 0; c < C; ++c) res_bound[c] = prm->res_factor * std::sqrt(res_bound[c]);
  // per sub-cube: sum over its channels of row k of the channel sums
  auto sub_sum = [&](int k, int c) {
    double v = 0.0;
    for (int l = c; l < L; l += C) v += h[static_cast<size_t>(k) * L + l];
    return v;
  };
  float *theta = const_cast<float *>(s->theta);
  double *theta_bar = const_cast<double *>(s->theta_bar);
  // Activity flags on the device: the kernels of a pass or an iteration
  // change only the sub-cubes still running (the others keep their state
  // bit for bit).  Uploaded when they change; the loop synchronises every
  // iteration, so the host copy is never rewritten while a copy is pending.
  int32_t *d_active = reinterpret_cast<int32_t *>(static_cast<char *>(p->ws) + p->ws_active);
  std::vector<int32_t> act(C, 0), uploaded(C, -1);
  auto upload = [&]() -> int {
    if (act == uploaded) return FHS_OK;
    if (hipMemcpyAsync(d_active, act.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, st) != hipSuccess)
      return fail(FHS_EHIP, "reweighting solve: uploading the sub-cube flags failed");
    uploaded = act;
    return FHS_OK;
  };
  std::vector<int32_t> outer(C, prm->max_reweights > 0 ? 1 : 0), pc(C, 0);
  std::vector<double> xi_c(C, kInf), res_c(C, 0.0), rw_c(C, kInf);
  std::vector<double> xi_h(C);
  fhs_solve_report rep{0, 0};
  if (iters)
    for (int64_t i = 0; i < static_cast<int64_t>(prm->max_reweights) * C; ++i) iters[i] = 0;
  if (rw_xi)
    for (int64_t i = 0; i < static_cast<int64_t>(prm->max_reweights) * C; ++i) rw_xi[i] = kInf;
  auto any = [](const std::vector<int32_t> &v) {
    for (int32_t e : v)
      if (e) return true;
    return false;
  };
  // Alg. 1 for every sub-cube c (its own pass counter t_c and relative
  // variation); the sub-cubes still in their loop advance together, one pass
  // at a time, so pass t is pass t of each of them.
  for (int t = 0; any(outer); ++t) {
    act = outer;
    if (int rc = upload()) return rc;
    if (int rc = reweight(p, s->x, upsilon, upsilon_bar, theta, theta_bar, stream, d_active)) return rc;
    if (hipMemcpyAsync(x_prev, s->x, cube_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->xcheck, s->x, cube_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(FHS_EHIP, "reweighting solve: device copy failed");
    // Alg. 2 from X_c(t) for each running sub-cube: its own p, xi_c and the
    // residual r_c of the iterate entering each iteration
    for (int c = 0; c < C; ++c) {
      pc[c] = 0;
      xi_c[c] = kInf;
    }
    for (int32_t it = 0; any(act); ++it) {
      if (int rc = channel_sums(p, s->y, s->x, h.data(), st)) return rc;
      for (int c = 0; c < C; ++c)
        if (act[c]) res_c[c] = std::sqrt(sub_sum(1, c));
      if (int rc = upload()) return rc;
      double *xi_dev = s->xi + static_cast<int64_t>(it) * C;
      if (int rc = iteration(p, s, xi_dev, stream, d_active)) return rc;
      if (hipMemcpyAsync(xi_h.data(), xi_dev, sizeof(double) * C, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(FHS_EHIP, "reweighting solve: reading xi failed");
      for (int c = 0; c < C; ++c) {
        if (!act[c]) continue;
        xi_c[c] = xi_h[c];
        ++pc[c];
        ++rep.iterations;
        act[c] = pc[c] < prm->min_iter ||
                 (pc[c] < prm->max_iter && (xi_c[c] > prm->pdfb_tol || res_c[c] > res_bound[c]));
      }
    }
    // relative variation of each sub-cube between reweights
    if (int rc = channel_sums(p, x_prev, s->x, h.data(), st)) return rc;
    for (int c = 0; c < C; ++c) {
      if (!outer[c]) continue;
      const double n0 = sub_sum(0, c);
      rw_c[c] = n0 > 0.0 ? std::sqrt(sub_sum(1, c) / n0) : kInf;
      if (iters) iters[static_cast<int64_t>(t) * C + c] = pc[c];
      if (rw_xi) rw_xi[static_cast<int64_t>(t) * C + c] = rw_c[c];
      outer[c] = t + 1 < prm->max_reweights && rw_c[c] > prm->rw_tol;
    }
    rep.runs = t + 1;
  }
  if (report) *report = rep;
  return FHS_OK;
}

int fhs_pdfb_graph_create(const fhs_plan *p, const fhs_pdfb_state *s, int32_t n_iter, fhs_graph **out) {
  if (!out) return fail(FHS_EINVAL, "fhs_pdfb_graph_create: null output");
  *out = nullptr;
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (int rc = check_state(s)) return rc;
  if (n_iter < 1) return fail(FHS_EINVAL, "n_iter must be >= 1");
  if (p->prof_kernel >= 0) return fail(FHS_EINVAL, "disable kernel profiling before capturing a graph");
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(FHS_EHIP, "hipStreamCreateWithFlags failed");
  auto *g = new (std::nothrow) fhs_graph;
  if (!g) {
    (void)hipStreamDestroy(cs);
    return fail(FHS_ENOMEM, "out of host memory");
  }
  int rc = FHS_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(FHS_EHIP, "hipStreamBeginCapture failed");
  } else {
    for (int32_t i = 0; i < n_iter && rc == FHS_OK; ++i) rc = fhs_pdfb_iteration(p, s, i, cs);
    const hipError_t e = hipStreamEndCapture(cs, &g->graph);
    if (rc == FHS_OK && e != hipSuccess) rc = fail(FHS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  if (rc == FHS_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = fail(FHS_EHIP, "hipGraphInstantiate failed");
  (void)hipStreamDestroy(cs);
  if (rc != FHS_OK) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return rc;
  }
  g->iterations = n_iter;
  *out = g;
  return FHS_OK;
}

int fhs_graph_launch(const fhs_graph *g, void *stream) {
  if (!g || !g->exec) return fail(FHS_EINVAL, "null graph");
  const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(FHS_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return FHS_OK;
}

void fhs_graph_destroy(fhs_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
