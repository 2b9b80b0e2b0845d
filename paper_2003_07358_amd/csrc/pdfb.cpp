// Whole PDFB iterations (Alg. 2) with the identity as measurement operator:
// the facet step, the data-fidelity dual, the primal update and the
// extrapolation, enqueued on one stream, and their capture into a HIP graph
// so that many iterations replay with one launch.
#include <hip/hip_runtime.h>

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
