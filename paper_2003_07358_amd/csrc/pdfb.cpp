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
            const float *grad, double tau, double *xi, void *stream) {
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
  a.tau = tau;
  a.npix = static_cast<int64_t>(p->cfg.ny) * p->cfg.nx;
  a.ppb = p->red_ppb;
  a.L = p->L;
  a.nblocks = p->red_blocks;
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
  if (int rc = check_state(s)) return rc;
  if (iter < 0) return fail(FHS_EINVAL, "iteration index must be >= 0");
  if (int rc = fhs_facet_prox_step(p, s->xcheck, s->p, s->w, s->theta, s->theta_bar, s->mu, s->mu_bar, s->zeta,
                                   s->kappa, s->grad, stream))
    return rc;
  return closure(p, s->x, s->xcheck, s->v, s->y, s->eps, s->grad, s->tau, s->xi + iter, stream);
}

int fhs_reweighting_solve(const fhs_plan *p, const fhs_pdfb_state *s, const double *upsilon,
                          const double *upsilon_bar, float *x_prev, const fhs_solve_params *prm, int32_t *iters,
                          fhs_solve_report *report, void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  if (int rc = check_state(s)) return rc;
  if (!upsilon || !upsilon_bar || !x_prev || !prm) return fail(FHS_EINVAL, "fhs_reweighting_solve: null argument");
  if (prm->max_reweights < 0 || prm->min_iter < 0 || prm->max_iter < 1 || prm->max_iter < prm->min_iter)
    return fail(FHS_EINVAL, "reweighting solve: need max_reweights >= 0 and 1 <= max_iter, min_iter <= max_iter");
  if (!(prm->rw_tol >= 0) || !(prm->pdfb_tol >= 0) || !(prm->res_factor > 0))
    return fail(FHS_EINVAL, "reweighting solve: tolerances must be >= 0 and res_factor > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int L = p->L;
  const size_t cube_bytes = static_cast<size_t>(p->cfg.ny) * p->cfg.nx * L * sizeof(float);
  std::vector<double> h(2 * static_cast<size_t>(L));
  // ||eps||
  if (hipMemcpyAsync(h.data(), s->eps, sizeof(double) * L, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(FHS_EHIP, "reweighting solve: reading eps failed");
  double eps2 = 0.0;
  for (int l = 0; l < L; ++l) eps2 += h[l] * h[l];
  const double res_bound = prm->res_factor * std::sqrt(eps2);
  auto sum_of = [&](int k) {
    double v = 0.0;
    for (int l = 0; l < L; ++l) v += h[static_cast<size_t>(k) * L + l];
    return v;
  };
  float *theta = const_cast<float *>(s->theta);
  double *theta_bar = const_cast<double *>(s->theta_bar);
  fhs_solve_report rep{0, 0, std::numeric_limits<double>::infinity(), std::numeric_limits<double>::infinity(),
                       std::numeric_limits<double>::infinity()};
  double rw_xi = std::numeric_limits<double>::infinity();
  for (int t = 0; t < prm->max_reweights && rw_xi > prm->rw_tol; ++t) {
    if (int rc = fhs_reweight(p, s->x, upsilon, upsilon_bar, theta, theta_bar, stream)) return rc;
    if (hipMemcpyAsync(x_prev, s->x, cube_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->xcheck, s->x, cube_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(FHS_EHIP, "reweighting solve: device copy failed");
    // Alg. 2 from X(t): r of the iterate entering each iteration
    if (int rc = channel_sums(p, s->y, s->x, h.data(), st)) return rc;
    double res = std::sqrt(sum_of(1)), xi = std::numeric_limits<double>::infinity();
    int32_t it = 0;
    while (it < prm->min_iter || (it < prm->max_iter && (xi > prm->pdfb_tol || res > res_bound))) {
      if (it > 0)
        if (int rc = channel_sums(p, s->y, s->x, h.data(), st)) return rc;
      res = std::sqrt(sum_of(1));
      if (int rc = fhs_pdfb_iteration(p, s, it, stream)) return rc;
      if (hipMemcpyAsync(&xi, s->xi + it, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(FHS_EHIP, "reweighting solve: reading xi failed");
      ++it;
    }
    if (iters) iters[t] = it;
    rep.iterations += it;
    rep.last_xi = xi;
    rep.last_res = res;
    // relative variation between reweights
    if (int rc = channel_sums(p, x_prev, s->x, h.data(), st)) return rc;
    const double n0 = sum_of(0);
    rw_xi = n0 > 0.0 ? std::sqrt(sum_of(1) / n0) : std::numeric_limits<double>::infinity();
    rep.runs = t + 1;
  }
  rep.rw_xi = rw_xi;
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
