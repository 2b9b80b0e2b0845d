// SARA analysis with the fused l21 dual update, for gfx950 (Sec. 2.3.1; Alg. 2
// l21 dual update; row shrink of Table 1).
//
// Transform: zero-extended expansive separable DWT, causal index convention
// a[k] = sum_m h[m] x[2k+1-m], k < floor((n+L-1)/2), along columns and rows,
// recursing on the low-low band; stored coefficients are divided by 3 (nine
// bases).  The faceted transform of Sec. 2.4.2 equals this global one, so the
// kernel tiles the global transform.
//
// Work decomposition: a workgroup owns TKX coefficient columns (all channel
// positions of a sub-cube on Lcp consecutive lanes) and a run of coefficient
// rows of one basis at one level.  It streams input rows top to bottom: step g
// filters input rows 2g, 2g+1 (relative to the first needed row) horizontally
// into a per-thread register ring, and once the ring holds NTAP rows filters
// vertically to emit one coefficient row of the four bands.
//
// Memory pipeline: steps are grouped into phases of P steps.  The 2P input row
// segments of a phase are copied HBM -> LDS by buffer loads with LDS
// destination one phase ahead (double-buffered LDS), and the W / theta values
// of each emitted row are loaded into registers one phase ahead, so a phase
// computes while the next phase's data is in flight; one barrier per phase.
//
// Precision: FP32 in / FP32 out, FP64 accumulation (detail coefficients are
// differences of large neighbouring values).
#include <hip/hip_runtime.h>

#include "fhs_filters.h"
#include "fhs_internal.h"
#include "lds_stage.h"

namespace fhs {

namespace {

constexpr double kThird = 1.0 / 3.0;  // 1 / sqrt(9): nine bases

// W and theta of the (up to four) bands of one emitted row.
struct EmitPre {
  float w[4], th[4];
};

// wrow = (ky Kx + kx) L + p and trow = c I + ky Kx + kx locate the row in band
// coordinates; band s adds off[s] L (resp. off[s]).
__device__ __forceinline__ void emit_prefetch(const AnaArgs &A, const AnaBand &B, bool valid, int64_t wrow,
                                              int64_t trow, EmitPre &e) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    e.w[s] = 0.0f;
    e.th[s] = 0.0f;
  }
  if (A.mode != 1 || !valid) return;
  const int ns = B.ll_out ? 3 : 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s < ns) {
      e.w[s] = A.w[wrow + B.off[s] * A.L];
      e.th[s] = A.theta[trow + B.off[s]];
    }
  }
}

// Writes / updates one coefficient (value already divided by 3): W element wi,
// theta element ti.
__device__ __forceinline__ void emit_coef(const AnaArgs &A, int64_t wi, int64_t ti, bool ok, int lane, float v,
                                          float thr, float wold, float th) {
  if (A.mode == 0) {
    if (ok) A.w[wi] = v;
  } else if (A.mode == 1) {
    // u = W_i + [Psi^dagger x]_i ; W_i <- u min(1, thr theta_i / ||u||), 0 if u = 0
    const float u = ok ? wold + v : 0.0f;
    const float r2 = seg_sum(u * u, A.Lcp);
    const float s = r2 > 0.0f ? fminf(1.0f, thr * th * __frsqrt_rn(r2)) : 0.0f;
    if (ok) A.w[wi] = u * s;
  } else {
    // theta_i = upsilon / (||[Psi^dagger x]_i|| + upsilon)
    const float vv = ok ? v : 0.0f;
    const float r2 = seg_sum(vv * vv, A.Lcp);
    if (ok && lane == 0) A.theta[ti] = thr / (sqrtf(r2) + thr);
  }
}

template <int NTAP, int P>
__device__ __forceinline__ void ana_basis(const AnaArgs &A, const AnaBand &B, int wg, float *smem) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % Lcp, grp = tid / Lcp, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? (B.in_natural ? c + lane * C : p) : 0;
  const int TKX = A.tkx1;
  const int strip = wg % B.strips, yb = wg / B.strips;
  const int kx0 = strip * TKX, ky0 = yb * A.tky;
  const int ky1 = min(ky0 + A.tky, B.Ky);
  const int segn = (2 * TKX + NTAP - 2) * L;  // floats of one input row segment
  const int segp = round_up(segn, 64);
  const int64_t rowlen = static_cast<int64_t>(B.in_nx) * L;
  const int64_t seg0 = static_cast<int64_t>(2 * kx0 + 2 - NTAP) * L;
  const int ystart = 2 * ky0 + 2 - NTAP;
  const int nsteps = (ky1 - ky0) + H - 1;
  const int nph = (nsteps + P - 1) / P;
  const int kx = kx0 + kq;
  const bool ok = lv && kx < B.Kx;
  float thr = 0.0f;
  if (A.mode == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (A.mode == 2) thr = static_cast<float>(A.mu[c]);

  // input rows of phase ph -> LDS buffer ph & 1 (2P segments, spread over waves)
  const int wv = wave_id(), nwv = full_wave_count();
  auto issue_phase = [&](int ph) {
    float *dst = smem + (ph & 1) * 2 * P * segp;
    if (wv >= nwv) return;
    for (int j = wv; j < 2 * P; j += nwv) {
      const int y = ystart + 2 * P * ph + j;
      const bool yv = y >= 0 && y < B.in_ny;
      wave_copy_row(B.in + (yv ? static_cast<int64_t>(y) * rowlen : 0), rowlen, seg0, segn, yv, dst + j * segp);
    }
  };

  // row locators of step g's output row ky = ky0 + g - (H-1)
  const int64_t KxL = static_cast<int64_t>(B.Kx) * L;
  const int64_t wrow0 = static_cast<int64_t>(ky0 - (H - 1)) * KxL + static_cast<int64_t>(kx) * L + p;
  const int64_t trow0 = static_cast<int64_t>(c) * A.I + static_cast<int64_t>(ky0 - (H - 1)) * B.Kx + kx;
  auto row_ok = [&](int g) {
    const int ky = ky0 + g - (H - 1);
    return ok && ky >= 0 && ky < B.Ky;
  };

  double rl[NTAP], rh[NTAP];
#pragma unroll
  for (int m = 0; m < NTAP; ++m) rl[m] = rh[m] = 0.0;
  EmitPre wq[P];
#pragma unroll
  for (int k = 0; k < P; ++k) emit_prefetch(A, B, row_ok(k), wrow0 + k * KxL, trow0 + k * B.Kx, wq[k]);
  issue_phase(0);

  for (int ph = 0; ph < nph; ++ph) {
    wait_loads_and_sync();
    if (ph + 1 < nph) issue_phase(ph + 1);
    const float *buf = smem + (ph & 1) * 2 * P * segp;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int g = ph * P + k;
      if (g < nsteps) {
        const EmitPre cur = wq[k];
        const int64_t wrow = wrow0 + g * KxL, trow = trow0 + static_cast<int64_t>(g) * B.Kx;
        emit_prefetch(A, B, row_ok(g + P), wrow + P * KxL, trow + P * B.Kx, wq[k]);
        // horizontal filter of the step's two rows into the ring (newest last)
#pragma unroll
        for (int m = 0; m + 2 < NTAP; ++m) {
          rl[m] = rl[m + 2];
          rh[m] = rh[m + 2];
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const float *bp = buf + (2 * k + r) * segp + (2 * kq + NTAP - 1) * L + chan;
          double sl = 0.0, sh = 0.0;
#pragma unroll
          for (int m = 0; m < NTAP; ++m) {
            const double v = static_cast<double>(bp[-m * L]);
            sl = fma(T::hd[m], v, sl);
            sh = fma(T::gd[m], v, sh);
          }
          rl[NTAP - 2 + r] = sl;
          rh[NTAP - 2 + r] = sh;
        }
        if (g >= H - 1) {
          // vertical filter: ring entry NTAP-1-m holds input row 2ky+1-m
          const int ky = ky0 + g - (H - 1);
          double ll = 0.0, lh = 0.0, hl = 0.0, hh = 0.0;
#pragma unroll
          for (int m = 0; m < NTAP; ++m) {
            ll = fma(T::hd[m], rl[NTAP - 1 - m], ll);
            lh = fma(T::hd[m], rh[NTAP - 1 - m], lh);
            hl = fma(T::gd[m], rl[NTAP - 1 - m], hl);
            hh = fma(T::gd[m], rh[NTAP - 1 - m], hh);
          }
          (void)ky;
          emit_coef(A, wrow + B.off[0] * L, trow + B.off[0], ok, lane, static_cast<float>(lh * kThird), thr,
                    cur.w[0], cur.th[0]);
          emit_coef(A, wrow + B.off[1] * L, trow + B.off[1], ok, lane, static_cast<float>(hl * kThird), thr,
                    cur.w[1], cur.th[1]);
          emit_coef(A, wrow + B.off[2] * L, trow + B.off[2], ok, lane, static_cast<float>(hh * kThird), thr,
                    cur.w[2], cur.th[2]);
          if (B.ll_out) {
            if (ok) B.ll_out[wrow] = static_cast<float>(ll);
          } else {
            emit_coef(A, wrow + B.off[3] * L, trow + B.off[3], ok, lane, static_cast<float>(ll * kThird), thr,
                      cur.w[3], cur.th[3]);
          }
        }
      }
    }
  }
  drain_loads();  // no LDS copy may land after the workgroup ends
}

// Dirac basis: coefficient row = pixel; grid-stride over pixels, 4 in flight.
__device__ __forceinline__ void ana_dirac(const AnaArgs &A, const AnaBand &B, int wg) {
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % Lcp, grp = tid / Lcp, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? c + lane * C : 0;
  constexpr int E = 4;
  const int64_t npix = static_cast<int64_t>(B.in_ny) * B.in_nx;
  const int64_t stride = static_cast<int64_t>(B.strips) * A.tkx1;  // strips = Dirac workgroups
  float thr = 0.0f;
  if (A.mode == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (A.mode == 2) thr = static_cast<float>(A.mu[c]);
  for (int64_t pix0 = static_cast<int64_t>(wg) * A.tkx1 + kq; pix0 - kq < npix; pix0 += E * stride) {
    float v[E], w[E], th[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t pix = pix0 + e * stride;
      const bool ok = lv && pix < npix;
      const int64_t i = B.off[0] + pix;
      v[e] = ok ? B.in[pix * L + chan] * (1.0f / 3.0f) : 0.0f;
      w[e] = (ok && A.mode == 1) ? A.w[i * L + p] : 0.0f;
      th[e] = (ok && A.mode == 1) ? A.theta[c * A.I + i] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t pix = pix0 + e * stride;
      const bool ok = lv && pix < npix;
      const int64_t i = B.off[0] + pix;
      emit_coef(A, i * L + p, static_cast<int64_t>(c) * A.I + i, ok, lane, v[e], thr, w[e], th[e]);
    }
  }
}

}  // namespace

// FIRST: level 1 (reads the cube, also updates the Dirac basis); a separate
// instantiation so that its launches are timed and profiled on their own.
template <bool FIRST, int P>
__global__ void __launch_bounds__(256) ana_kernel(AnaArgs A) {
  extern __shared__ float smem[];
  const int id = blockIdx.x;
  int b = 0;
  while (b < kBases && id >= A.wg_prefix[b + 1]) ++b;
  const int wg = id - A.wg_prefix[b];
  switch (b) {
    case 0: ana_basis<2, P>(A, A.b[0], wg, smem); break;
    case 1: ana_basis<4, P>(A, A.b[1], wg, smem); break;
    case 2: ana_basis<6, P>(A, A.b[2], wg, smem); break;
    case 3: ana_basis<8, P>(A, A.b[3], wg, smem); break;
    case 4: ana_basis<10, P>(A, A.b[4], wg, smem); break;
    case 5: ana_basis<12, P>(A, A.b[5], wg, smem); break;
    case 6: ana_basis<14, P>(A, A.b[6], wg, smem); break;
    case 7: ana_basis<16, P>(A, A.b[7], wg, smem); break;
    default:
      if (FIRST) ana_dirac(A, A.b[8], wg);
      break;
  }
}

// Steps per phase: 4, or 2 when four would need more than 64 KB of LDS.
int analysis_phase(int tkx1, int L) {
  const int segp = ((2 * tkx1 + kMaxTap - 2) * L + 63) / 64 * 64;
  return 2 * 2 * 4 * segp * 4 <= 65536 ? 4 : 2;
}

int launch_analysis(const AnaArgs &a, int nthreads, bool first, void *stream) {
  const int nwg = a.wg_prefix[kBases + 1];
  if (nwg <= 0) return FHS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int P = analysis_phase(a.tkx1, a.L);
  const int segp = ((2 * a.tkx1 + kMaxTap - 2) * a.L + 63) / 64 * 64;
  const size_t lds = static_cast<size_t>(2 * 2 * P * segp) * sizeof(float);
  if (P == 4) {
    if (first)
      hipLaunchKernelGGL((ana_kernel<true, 4>), dim3(nwg), dim3(nthreads), lds, s, a);
    else
      hipLaunchKernelGGL((ana_kernel<false, 4>), dim3(nwg), dim3(nthreads), lds, s, a);
  } else {
    if (first)
      hipLaunchKernelGGL((ana_kernel<true, 2>), dim3(nwg), dim3(nthreads), lds, s, a);
    else
      hipLaunchKernelGGL((ana_kernel<false, 2>), dim3(nwg), dim3(nthreads), lds, s, a);
  }
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("analysis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

}  // namespace fhs
