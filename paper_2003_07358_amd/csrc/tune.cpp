// Autotuner of the launch shapes (fhs_plan_autotune): coordinate descent over
// the fields of fhs_tuning, each candidate timed on whole facet steps with
// HIP events on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fhs_internal.h"

using namespace fhs;

namespace {

struct Step {
  const float *x;
  float *p, *w;
  const float *theta;
  const double *theta_bar, *mu, *mu_bar;
  float *grad;
};

// Mean ms of `reps` steps (after one untimed step); < 0 on failure.
float time_steps(fhs_plan *p, const Step &a, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  auto one = [&]() {
    return fhs_facet_prox_step(p, a.x, a.p, a.w, a.theta, a.theta_bar, a.mu, a.mu_bar, 1.0, 1.0, a.grad, s);
  };
  if (one() != FHS_OK) return -1.0f;
  if (hipEventRecord(e0, s) != hipSuccess) return -1.0f;
  for (int r = 0; r < reps; ++r)
    if (one() != FHS_OK) return -1.0f;
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0f;
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
  return ms / reps;
}

}  // namespace

extern "C" int fhs_plan_autotune(fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                                 const double *theta_bar, const double *mu, const double *mu_bar, float *grad,
                                 int32_t reps, void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!p->ws) return fail(FHS_ENOWORKSPACE, "no workspace attached (fhs_plan_set_workspace)");
  if (reps < 1) return fail(FHS_EINVAL, "reps must be >= 1");
  if (p->prof_kernel >= 0) return fail(FHS_EINVAL, "disable kernel profiling before autotuning");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(FHS_EHIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(FHS_EHIP, "hipEventCreate failed");
  }
  const Step a{xcheck, pdual, w, theta, theta_bar, mu, mu_bar, grad};
  fhs_tuning best = p->tune;
  float best_ms = time_steps(p, a, reps, s, e0, e1);
  int rc = best_ms < 0 ? FHS_EHIP : FHS_OK;
  // try one candidate: keep it if valid and faster
  auto trial = [&](const fhs_tuning &cand) {
    if (rc != FHS_OK) return;
    if (fhs_plan_set_tuning(p, &cand) != FHS_OK) {
      (void)fhs_plan_set_tuning(p, &best);
      return;
    }
    const float ms = time_steps(p, a, reps, s, e0, e1);
    if (ms < 0) {
      rc = FHS_EHIP;
    } else if (ms < best_ms) {
      best_ms = ms;
      best = cand;
    }
    (void)fhs_plan_set_tuning(p, &best);
  };
  // two passes of coordinate descent (the fields interact: the second pass
  // revisits each with the others settled); the second is skipped if the
  // first changed nothing
  for (int pass = 0; pass < 2; ++pass) {
    const float pass_start = best_ms;
    // the step's structure first (the two streams' balance), then the shapes
    for (int conc : {0, 1}) {
      fhs_tuning c = best;
      c.concurrent = conc;
      trial(c);
    }
    const int ch0 = p->nuc_chunk_min * 2;  // (the default chunk)
    for (int f : {1, 2, 4, 8, 16}) {
      fhs_tuning c = best;
      c.nuc_chunk_rows = std::max(p->nuc_chunk_min, ch0 * f / 2);
      trial(c);
    }
    for (int seg : {16, 32, 64}) {
      fhs_tuning c = best;
      c.nuc_seg = seg;
      trial(c);
    }
    for (int j = 0; j < p->cfg.levels && j < kMaxLevels; ++j) {
      for (int d : {0, 1}) {
        fhs_tuning c = best;
        c.ana_direct = (best.ana_direct & ~(1 << j)) | (d << j);
        trial(c);
      }
      for (int o : {0, 1}) {
        fhs_tuning c = best;
        c.ana_order = (best.ana_order & ~(1 << j)) | (o << j);
        trial(c);
      }
      for (int rows : {8, 16, 32, 64, 128}) {
        fhs_tuning c = best;
        c.ana_rows[j] = rows;
        trial(c);
      }
    }
    for (int ph : {1, 2, 4}) {
      fhs_tuning c = best;
      c.ana_phase = ph;
      trial(c);
    }
    for (int rows : {32, 64, 128}) {
      fhs_tuning c = best;
      c.syn_rows = rows;
      trial(c);
    }
    for (int rows : {64, 128, 256}) {
      fhs_tuning c = best;
      c.fin_rows = rows;
      trial(c);
    }
    for (int waves : {4, 6, 8}) {
      fhs_tuning c = best;
      c.fin_waves = waves;
      trial(c);
    }
    if (best_ms == pass_start) break;
  }
  (void)fhs_plan_set_tuning(p, &best);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != FHS_OK) return fail(rc, "autotune: a timed step failed");
  return FHS_OK;
}
