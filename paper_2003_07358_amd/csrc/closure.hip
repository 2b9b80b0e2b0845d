// The rest of a PDFB iteration around the facet step, for gfx950 (Alg. 2):
// the data-fidelity dual update with the identity as measurement operator
// (projection onto the l2 ball of Table 1, U = I, eta = 1), the primal update
// (projection onto the non-negative orthant, Table 1), the extrapolation and
// the relative variation of the iterate.  Elementwise HBM-bound passes plus
// per-channel and global sums, reduced in a fixed order so that results are
// bitwise reproducible run to run.
//
//   closure_norm   : per block and channel l, sum over its pixels of
//                    d^2, d = v + xcheck - y                     (FP64)
//   closure_factor : f_l = max(0, 1 - eps_l / ||d_l||)  (0 if ||d_l|| = 0),
//                    so that (I - proj_B(y_l, eps_l))(v + xcheck) = f_l d
//   closure_primal : v <- f_l d;  x+ = max(0, x - tau (grad + v));
//                    xcheck <- 2 x+ - x;  x <- x+; per block and channel
//                    the sums of (x+ - x)^2 and x^2               (FP64)
//   closure_xi     : per spectral sub-cube c (channels c, c + C, ...; Alg. 2
//                    solves each sub-problem on its own)
//                    xi_c = ||x+_c - x_c||_F / ||x_c||_F (+inf if x_c = 0)
//
// With activity flags, the channels of a frozen sub-cube are read but not
// written (its sums still come out, and are ignored by the caller).
//
// Thread layout: a block of 256 threads holds G = floor(256 / L) pixel groups
// of L threads; thread (g, l) always works on channel l, so the channel sums
// need no atomics.  Block b owns pixels [b * ppb, min((b + 1) * ppb, N)).
#include <hip/hip_runtime.h>

#include "fhs_internal.h"

namespace fhs {

namespace {

constexpr int kThreads = 256;

// Fixed-order sum over the G groups of each channel held in sh[g * L + l];
// thread l < L returns the sum for channel l.
__device__ __forceinline__ double group_sum(const double *sh, int G, int L, int l) {
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += sh[g * L + l];
  return s;
}

__global__ void __launch_bounds__(kThreads) closure_norm(ClosureArgs a) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int L = a.L, G = kThreads / L;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * a.ppb;
  const int64_t p1 = min(p0 + a.ppb, a.npix);
  double acc = 0.0;
  if (t < G * L) {
    const int g = t / L, l = t - (t / L) * L;
    for (int64_t p = p0 + g; p < p1; p += G) {
      const int64_t e = p * L + l;
      const double d = static_cast<double>(a.v[e]) + static_cast<double>(a.xcheck[e]) - static_cast<double>(a.y[e]);
      acc += d * d;
    }
  }
  sh[t] = acc;
  __syncthreads();
  if (t < L) a.part[static_cast<int64_t>(blockIdx.x) * L + t] = group_sum(sh, G, L, t);
}

// One block: channel l's partials are split over the G groups of the block
// (group g sums blocks g, g + G, ...), then the groups are summed in order.
__global__ void __launch_bounds__(kThreads) closure_factor(ClosureArgs a) {
  __shared__ double sh[kThreads];
  const int t = threadIdx.x;
  const int L = a.L, G = kThreads / L;
  double acc = 0.0;
  if (t < G * L) {
    const int g = t / L, l = t - (t / L) * L;
    for (int b = g; b < a.nblocks; b += G) acc += a.part[static_cast<int64_t>(b) * L + l];
  }
  sh[t] = acc;
  __syncthreads();
  if (t < L) {
    const double nrm = sqrt(group_sum(sh, G, L, t));
    const double eps = a.eps[t];
    a.factor[t] = nrm > eps ? 1.0 - eps / nrm : 0.0;
  }
}

__global__ void __launch_bounds__(kThreads) closure_primal(ClosureArgs a) {
  __shared__ double sh0[kThreads], sh1[kThreads];
  const int t = threadIdx.x;
  const int L = a.L, G = kThreads / L;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * a.ppb;
  const int64_t p1 = min(p0 + a.ppb, a.npix);
  double dx2 = 0.0, x2 = 0.0;
  if (t < G * L) {
    const int g = t / L, l = t - (t / L) * L;
    // channel l belongs to sub-cube l mod C (l / L_c for contiguous blocks);
    // a frozen sub-cube keeps x, xcheck, v
    const bool act = a.active == nullptr || a.active[a.contig ? l / (L / a.C) : l % a.C] != 0;
    const double f = a.factor[l];
    const double tau = a.tau;
    for (int64_t p = p0 + g; p < p1; p += G) {
      const int64_t e = p * L + l;
      const double xo = a.x[e];
      const double d = static_cast<double>(a.v[e]) + static_cast<double>(a.xcheck[e]) - static_cast<double>(a.y[e]);
      const double vn = f * d;
      const double xn = fmax(0.0, xo - tau * (static_cast<double>(a.grad[e]) + vn));
      if (act) {
        a.v[e] = static_cast<float>(vn);
        a.x[e] = static_cast<float>(xn);
        a.xcheck[e] = static_cast<float>(2.0 * xn - xo);
      }
      dx2 += (xn - xo) * (xn - xo);
      x2 += xo * xo;
    }
  }
  sh0[t] = dx2;
  sh1[t] = x2;
  __syncthreads();
  // per channel: the block's sums of (x+ - x)^2 and x^2, groups in order
  if (t < L) {
    a.part[static_cast<int64_t>(blockIdx.x) * 2 * L + t] = group_sum(sh0, G, L, t);
    a.part[static_cast<int64_t>(blockIdx.x) * 2 * L + L + t] = group_sum(sh1, G, L, t);
  }
}

// One block: per channel, the block partials (split over the G groups, then
// the groups in order); per sub-cube c, its channels c, c + C, ... in order;
// xi_c = sqrt(sum (x+ - x)^2 / sum x^2) (+inf if x_c = 0).
__global__ void __launch_bounds__(kThreads) closure_xi(ClosureArgs a) {
  __shared__ double sh0[kThreads], sh1[kThreads];
  __shared__ double ch0[kThreads], ch1[kThreads];
  const int t = threadIdx.x;
  const int L = a.L, G = kThreads / L;
  double s0 = 0.0, s1 = 0.0;
  if (t < G * L) {
    const int g = t / L, l = t - (t / L) * L;
    for (int b = g; b < a.nblocks; b += G) {
      s0 += a.part[static_cast<int64_t>(b) * 2 * L + l];
      s1 += a.part[static_cast<int64_t>(b) * 2 * L + L + l];
    }
  }
  sh0[t] = s0;
  sh1[t] = s1;
  __syncthreads();
  if (t < L) {
    ch0[t] = group_sum(sh0, G, L, t);
    ch1[t] = group_sum(sh1, G, L, t);
  }
  __syncthreads();
  if (t < a.C) {
    double a0 = 0.0, a1 = 0.0;
    const int l0 = a.contig ? t * (L / a.C) : t, l1 = a.contig ? l0 + L / a.C : L, dl = a.contig ? 1 : a.C;
    for (int l = l0; l < l1; l += dl) {
      a0 += ch0[l];
      a1 += ch1[l];
    }
    a.xi[t] = a1 > 0.0 ? sqrt(a0 / a1) : __builtin_huge_val();
  }
}

// Reconstruction metrics (Sec. 4.3): per block and channel the four sums
// sum r^2, sum (r - x)^2 and, with noise levels, the same of
// a = log10(r / eps + 1), b = log10(x / eps + 1); then one block sums the
// partials in a fixed order and writes 10 log10(num / den) per channel.
__global__ void __launch_bounds__(kThreads) snr_part(SnrArgs a) {
  __shared__ double sh[4][kThreads];
  const int t = threadIdx.x;
  const int L = a.L, G = kThreads / L;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * a.ppb;
  const int64_t p1 = min(p0 + a.ppb, a.npix);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (t < G * L) {
    const int g = t / L, l = t - (t / L) * L;
    const double eps = a.eps ? a.eps[l] : 1.0;
    for (int64_t p = p0 + g; p < p1; p += G) {
      const int64_t e = p * L + l;
      const double r = a.ref[e], x = a.x[e];
      s[0] += r * r;
      s[1] += (r - x) * (r - x);
      if (a.eps) {
        const double lr = log10(r / eps + 1.0), lx = log10(x / eps + 1.0);
        s[2] += lr * lr;
        s[3] += (lr - lx) * (lr - lx);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][t] = s[k];
  __syncthreads();
  if (t < L)
#pragma unroll
    for (int k = 0; k < 4; ++k) a.part[(static_cast<int64_t>(blockIdx.x) * 4 + k) * L + t] = group_sum(sh[k], G, L, t);
}

__device__ __forceinline__ double db(double num, double den) {
  return den > 0.0 ? 10.0 * log10(num / den) : __builtin_huge_val();
}

__global__ void __launch_bounds__(kThreads) snr_final(SnrArgs a) {
  __shared__ double sh[4][kThreads];
  const int t = threadIdx.x;
  const int L = a.L, G = kThreads / L;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (t < G * L) {
    const int g = t / L, l = t - (t / L) * L;
    for (int b = g; b < a.nblocks; b += G)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] += a.part[(static_cast<int64_t>(b) * 4 + k) * L + l];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][t] = s[k];
  __syncthreads();
  if (t < L) {
    const double s0 = group_sum(sh[0], G, L, t), s1 = group_sum(sh[1], G, L, t);
    if (a.snr) a.snr[t] = db(s0, s1);
    if (a.sums) {
      a.sums[t] = s0;
      a.sums[L + t] = s1;
    }
    if (a.eps) a.snr_log[t] = db(group_sum(sh[2], G, L, t), group_sum(sh[3], G, L, t));
  }
}

int check(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string(what) + ": " + hipGetErrorString(err));
  return FHS_OK;
}

}  // namespace

int launch_snr(const SnrArgs &a, void *stream) {
  if (a.L < 1 || a.L > kThreads) return fail(FHS_EUNSUPPORTED, "snr: channels must be in [1, 256]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(snr_part, dim3(static_cast<unsigned>(a.nblocks)), dim3(kThreads), 0, s, a);
  if (int rc = check("snr_part")) return rc;
  hipLaunchKernelGGL(snr_final, dim3(1), dim3(kThreads), 0, s, a);
  return check("snr_final");
}

int launch_closure(const ClosureArgs &a, void *stream) {
  if (a.L < 1 || a.L > kThreads) return fail(FHS_EUNSUPPORTED, "closure: channels must be in [1, 256]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(a.nblocks)), block(kThreads);
  hipLaunchKernelGGL(closure_norm, grid, block, 0, s, a);
  if (int rc = check("closure_norm")) return rc;
  hipLaunchKernelGGL(closure_factor, dim3(1), block, 0, s, a);
  if (int rc = check("closure_factor")) return rc;
  hipLaunchKernelGGL(closure_primal, grid, block, 0, s, a);
  if (int rc = check("closure_primal")) return rc;
  hipLaunchKernelGGL(closure_xi, dim3(1), block, 0, s, a);
  return check("closure_xi");
}

}  // namespace fhs
