// SARA analysis with the fused l21 dual update, for gfx950 (Sec. 2.3.1; Alg. 2
// l21 dual update; row shrink of Table 1).  Device code, included by one
// translation unit per mode.
//
// Transform: zero-extended expansive separable DWT, causal index convention
// a[k] = sum_m h[m] x[2k+1-m], k < floor((n+L-1)/2), along columns and rows,
// recursing on the low-low band; stored coefficients are divided by 3 (nine
// bases).  The faceted transform of Sec. 2.4.2 equals this global one, so the
// kernel tiles the global transform.
//
// Work decomposition: a workgroup owns TKX coefficient columns (all channel
// positions of every sub-cube, LCP lanes per sub-cube) and a run of
// coefficient rows of one basis at one level.  It streams input rows top to
// bottom: step g filters input rows 2g, 2g+1 (relative to the first needed row)
// horizontally into a per-thread FP64 register ring, and once the ring holds
// NTAP rows filters vertically to emit one coefficient row of the four bands.
//
// Memory pipeline: steps are grouped into phases of P steps.  Per phase, the
// 2P input row segments and the W / theta values of the P emitted rows are
// copied HBM -> LDS by buffer loads whose destination is LDS, one phase ahead
// into a double buffer; one barrier per phase.  A row segment is one
// contiguous run of HBM ([column][channel]), copied as is.
//
// Launch order is XCD-aware: workgroup id -> XCD id % 8; each XCD walks a
// contiguous run of tiles and, for each tile, the 8 bases one after the other,
// so the input segments of a tile are fetched from HBM once per XCD L2.
//
// Precision: FP32 in / FP32 out, FP64 accumulation (detail coefficients are
// differences of large neighbouring values).
#pragma once

#include <hip/hip_runtime.h>

#include "fhs_filters.h"
#include "fhs_internal.h"
#include "lds_stage.h"

namespace fhs {
namespace ana {

constexpr double kThird = 1.0 / 3.0;  // 1 / sqrt(9): nine bases
constexpr int kMaxPhase = 4;          // steps per LDS phase, upper bound (the launch picks P)

typedef __attribute__((address_space(3))) unsigned int lds_u32;

__device__ __forceinline__ lds_u32 *lds_ptr(const float *p) {
  return reinterpret_cast<lds_u32 *>(reinterpret_cast<uintptr_t>(p));
}

// W_i <- u min(1, thr theta_i / ||u||) (0 if u = 0), u = W_i + v; returns the
// new value.  Segment sum over the LCP lanes of one coefficient row.
// (r2 = 0 gives rsq = inf and fminf(1, inf or NaN) = 1, so u * 1 = 0: no
// separate zero test is needed)
template <int LCP>
__device__ __forceinline__ float shrink(float u, float thr_th) {
  const float r2 = seg_sum(u * u, LCP);
  return u * fminf(1.0f, thr_th * __frsqrt_rn(r2));
}

template <int NTAP, int MODE, int LCP>
__device__ __forceinline__ void basis(const AnaArgs &A, const AnaBand &B, int tile, float *smem) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
  if (tile >= B.strips * B.yblocks) return;
  const int L = A.L, C = A.C, Lc = A.Lc, P = A.P;
  const int tid = threadIdx.x;
  const int lane = tid % LCP, grp = tid / LCP, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? (B.in_natural ? c + lane * C : p) : 0;
  const int TKX = A.tkx1;
  const int strip = tile % B.strips, yb = tile / B.strips;
  const int kx0 = B.kx_begin + strip * TKX, ky0 = B.ky_begin + yb * A.tky;
  const int ky1 = min(ky0 + A.tky, B.ky_end);
  const int kx = kx0 + kq;
  const bool ok = lv && kx < B.kx_end;
  const int NC = 2 * TKX + NTAP - 2;        // input columns of a row segment
  const int ROW = A.lds_row;                // LDS words per staged input row
  const int col0 = 2 * kx0 + 2 - NTAP;      // first input column
  const int ystart = 2 * ky0 + 2 - NTAP;
  const int nsteps = (ky1 - ky0) + H - 1;
  const int nph = (nsteps + P - 1) / P;
  const int64_t rowlen = static_cast<int64_t>(B.in_nx) * L;
  const int KxL = B.Kx * L;
  float thr = 0.0f;
  if (MODE == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (MODE == 2) thr = static_cast<float>(A.mu[c]);

  // ---- copy plan (per lane, fixed for the workgroup)
  const int wv = wave_id(), nwv = full_wave_count();
  const int ln = threadIdx.x & 63;
  const int64_t seg0 = static_cast<int64_t>(col0) * L;  // first float of a row segment
  const int segn = NC * L;                               // floats of a row segment
  // theta gather: word i = 64 j + ln -> (sub-cube i / TKX, column kx0 + i % TKX); C * TKX <= 128
  int th_voff[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = 64 * j + ln, cc = i / TKX, kk = i - cc * TKX;
    th_voff[j] = (cc < C && kx0 + kk < B.kx_end) ? static_cast<int>((static_cast<int64_t>(cc) * A.I + kx0 + kk) * 4)
                                             : static_cast<int>(0x80000000u);
  }
  const int nth_chunks = (C * TKX + 63) / 64;

  auto issue_phase = [&](int ph) __attribute__((always_inline)) {
    if (wv >= nwv) return;
    float *buf = smem + (ph & 1) * A.lds_buf;
    const int ntask = 2 * P + (MODE == 1 ? 4 * P : 0);
    for (int t = wv; t < ntask; t += nwv) {
      if (t < 2 * P) {
        const int y = ystart + 2 * P * ph + t;
        const bool yv = y >= 0 && y < B.in_ny;
        wave_copy_row(B.in + (yv ? static_cast<int64_t>(y) * rowlen : 0), rowlen, seg0, segn, yv, buf + t * ROW);
      } else {
        const int k = (t - 2 * P) >> 2, s = (t - 2 * P) & 3;
        const int g = P * ph + k;
        const int ky = ky0 + g - (H - 1);
        // (explicit select: a dynamic index into the band descriptor would copy it to scratch)
        const int64_t boff = s == 0 ? B.off[0] : s == 1 ? B.off[1] : s == 2 ? B.off[2] : B.off[3];
        if (g >= nsteps || ky < 0 || ky >= B.Ky || boff < 0) continue;
        const int64_t rowi = boff + static_cast<int64_t>(ky) * B.Kx + kx0;  // first coefficient row
        // W of the TKX coefficient rows: TKX * L contiguous floats
        const int nw = min(TKX, B.kx_end - kx0) * L;
        const fhs_int32x4 wr = buffer_rsrc(A.w + rowi * L, static_cast<unsigned>(nw * 4));
        float *wdst = buf + A.lds_wv + (4 * k + s) * A.wpad;
        for (int j = 0; j < A.wpad; j += 64)
          fhs_raw_buffer_load_lds(wr, lds_ptr(wdst + j), 4, (j + ln) * 4, 0, 0, 0);
        // theta of the same rows for every sub-cube: a gather
        const fhs_int32x4 tr = buffer_rsrc(A.theta, static_cast<unsigned>(A.theta_bytes));
        float *tdst = buf + A.lds_th + (4 * k + s) * A.tpad;
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (j < nth_chunks)
            fhs_raw_buffer_load_lds(tr, lds_ptr(tdst + 64 * j), 4, th_voff[j],
                                    static_cast<int>((boff + static_cast<int64_t>(ky) * B.Kx) * 4), 0, 0);
      }
    }
  };

  double rl[NTAP], rh[NTAP];
#pragma unroll
  for (int m = 0; m < NTAP; ++m) rl[m] = rh[m] = 0.0;
  // LDS word of tap NTAP-1 (the lowest column) of this lane in an input row
  const int lbase = 2 * kq * L + chan;
  const int wl = kq * L + p;                 // lane's word in a W row segment
  const int tl = c * TKX + kq;               // lane's word in a theta segment

  issue_phase(0);
  for (int ph = 0; ph < nph; ++ph) {
    wait_loads_and_sync();
    if (ph + 1 < nph) issue_phase(ph + 1);
    const float *buf = smem + (ph & 1) * A.lds_buf;
#pragma unroll
    for (int k = 0; k < kMaxPhase; ++k) {
      const int g = ph * P + k;
      if (k < P && g < nsteps) {
        // horizontal filter of the step's two rows; the ring shifts by two
        // (entry NTAP-1-m holds input row 2g+1-m once filled)
#pragma unroll
        for (int m = 0; m + 2 < NTAP; ++m) {
          rl[m] = rl[m + 2];
          rh[m] = rh[m + 2];
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          // taps: h / 3 (the dictionary's 1/3 applied here), and g[m] =
          // (-1)^m h[NTAP-1-m] written with the sign on the data, so that only
          // NTAP distinct constants are live
          const float *bp = buf + (2 * k + r) * ROW + lbase;
          double sl = 0.0, sh = 0.0;
#pragma unroll
          for (int m = 0; m < NTAP; ++m) {
            const double v = static_cast<double>(bp[(NTAP - 1 - m) * L]);
            sl = fma(T::hd[m] * kThird, v, sl);
            sh = fma(T::hd[NTAP - 1 - m] * kThird, (m & 1) ? -v : v, sh);
          }
          rl[NTAP - 2 + r] = sl;
          rh[NTAP - 2 + r] = sh;
        }
        if (g >= H - 1) {
          // (the ring holds rows already divided by 3)
          double ll = 0.0, lh = 0.0, hl = 0.0, hh = 0.0;
#pragma unroll
          for (int m = 0; m < NTAP; ++m) {
            const double a = rl[NTAP - 1 - m], b = rh[NTAP - 1 - m];
            ll = fma(T::hd[m], a, ll);
            lh = fma(T::hd[m], b, lh);
            hl = fma(T::hd[NTAP - 1 - m], (m & 1) ? -a : a, hl);
            hh = fma(T::hd[NTAP - 1 - m], (m & 1) ? -b : b, hh);
          }
          const int ky = ky0 + g - (H - 1);
          const float vb[4] = {static_cast<float>(lh), static_cast<float>(hl), static_cast<float>(hh),
                               static_cast<float>(ll)};
          const bool last = B.ll_out == nullptr;
#pragma unroll
          for (int sb = 0; sb < 4; ++sb) {
            if (sb == 3 && !last) continue;
            const int64_t rowi = B.off[sb] + static_cast<int64_t>(ky) * B.Kx + kx0;
            float *wrow = A.w + rowi * L;
            if (MODE == 0) {
              if (ok) wrow[wl] = vb[sb];
            } else if (MODE == 1) {
              const float wold = buf[A.lds_wv + (4 * k + sb) * A.wpad + wl];
              const float th = buf[A.lds_th + (4 * k + sb) * A.tpad + tl];
              const float u = ok ? wold + vb[sb] : 0.0f;
              const float wn = shrink<LCP>(u, thr * th);
              if (ok) wrow[wl] = wn;
            } else {
              const float vv = ok ? vb[sb] : 0.0f;
              const float r2 = seg_sum(vv * vv, LCP);
              if (ok && lane == 0) A.theta[static_cast<int64_t>(c) * A.I + rowi + kq] = thr / (sqrtf(r2) + thr);
            }
          }
          if (B.ll_out && ok)
            B.ll_out[static_cast<int64_t>(ky) * KxL + static_cast<int64_t>(kx) * L + p] = static_cast<float>(3.0 * ll);
        }
      }
    }
  }
  drain_loads();  // no LDS copy may land after the workgroup ends
}

// The same computation without LDS: every lane loads its own filter taps and
// W / theta straight from HBM (through the caches) one step ahead into
// registers, with range-checked buffer loads (out-of-range columns and rows
// read as zero).  No barriers; the compiler's wait counts track each load, so
// stores never stall a step.
__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

template <int NTAP, int MODE, int LCP>
__device__ __forceinline__ void basis_direct(const AnaArgs &A, const AnaBand &B, int tile) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
  if (tile >= B.strips * B.yblocks) return;
  const int L = A.L, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % LCP, grp = tid / LCP, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? (B.in_natural ? c + lane * C : p) : 0;
  const int TKX = A.tkx1;
  const int strip = tile % B.strips, yb = tile / B.strips;
  const int kx0 = B.kx_begin + strip * TKX, ky0 = B.ky_begin + yb * A.tky;
  const int ky1 = min(ky0 + A.tky, B.ky_end);
  const int kx = kx0 + kq;
  const bool ok = lv && kx < B.kx_end;
  const int ystart = 2 * ky0 + 2 - NTAP;
  const int nsteps = (ky1 - ky0) + H - 1;
  const int64_t rowlen = static_cast<int64_t>(B.in_nx) * L;
  float thr = 0.0f;
  if (MODE == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (MODE == 2) thr = static_cast<float>(A.mu[c]);
  // byte offset of tap NTAP-1 (column 2 kx + 2 - NTAP) of this lane in a row;
  // tap m adds (NTAP-1-m) L 4 (negative columns wrap to huge offsets: zeros,
  // as do columns past the row)
  const int vbase = ((2 * kx + 2 - NTAP) * L + chan) * 4;
  const bool last = B.ll_out == nullptr;
  const __amdgpu_buffer_rsrc_t thr_r =
      __builtin_amdgcn_make_buffer_rsrc(A.theta, static_cast<short>(0), static_cast<int>(A.theta_bytes), 0x00020000);

  auto load_rows = [&](int g, float (&t)[2][NTAP]) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int y = ystart + 2 * g + r;
      const bool yv = g < nsteps && y >= 0 && y < B.in_ny;
      const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(B.in) + (yv ? static_cast<int64_t>(y) * rowlen : 0), static_cast<short>(0),
          yv ? static_cast<int>(rowlen * 4) : 0, 0x00020000);
#pragma unroll
      // (the whole offset in voffset: the range check does not see soffset)
      for (int m = 0; m < NTAP; ++m) t[r][m] = ld_f32(rr, vbase + (NTAP - 1 - m) * L * 4, 0);
    }
  };
  // W and theta of the row emitted at step g (mode 1)
  auto load_emit = [&](int g, float (&w)[4], float (&th)[4]) __attribute__((always_inline)) {
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      w[sb] = th[sb] = 0.0f;
      if (MODE == 1) {
        const int ky = ky0 + g - (H - 1);
        const bool v = ok && g < nsteps && ky >= ky0 && (sb < 3 || last);
        if (v) {
          const int64_t rowi = B.off[sb] + static_cast<int64_t>(ky) * B.Kx + kx;
          w[sb] = A.w[rowi * L + p];
          th[sb] = ld_f32(thr_r, static_cast<int>((static_cast<int64_t>(c) * A.I + rowi) * 4), 0);
        }
      }
    }
  };

  double rl[NTAP], rh[NTAP];
#pragma unroll
  for (int m = 0; m < NTAP; ++m) rl[m] = rh[m] = 0.0;
  float ta[2][NTAP], tb[2][NTAP];
  float wa[4], tha[4], wb[4], thb[4];
  load_rows(0, ta);
  load_emit(0, wa, tha);

  auto step = [&](int g, const float (&t)[2][NTAP], const float (&w)[4], const float (&th)[4])
      __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m + 2 < NTAP; ++m) {
      rl[m] = rl[m + 2];
      rh[m] = rh[m + 2];
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      double sl = 0.0, sh = 0.0;
#pragma unroll
      for (int m = 0; m < NTAP; ++m) {
        const double v = static_cast<double>(t[r][m]);
        sl = fma(T::hd[m] * kThird, v, sl);
        sh = fma(T::hd[NTAP - 1 - m] * kThird, (m & 1) ? -v : v, sh);
      }
      rl[NTAP - 2 + r] = sl;
      rh[NTAP - 2 + r] = sh;
    }
    if (g >= H - 1) {
      double ll = 0.0, lh = 0.0, hl = 0.0, hh = 0.0;
#pragma unroll
      for (int m = 0; m < NTAP; ++m) {
        const double a = rl[NTAP - 1 - m], b = rh[NTAP - 1 - m];
        ll = fma(T::hd[m], a, ll);
        lh = fma(T::hd[m], b, lh);
        hl = fma(T::hd[NTAP - 1 - m], (m & 1) ? -a : a, hl);
        hh = fma(T::hd[NTAP - 1 - m], (m & 1) ? -b : b, hh);
      }
      const int ky = ky0 + g - (H - 1);
      const float vb[4] = {static_cast<float>(lh), static_cast<float>(hl), static_cast<float>(hh),
                           static_cast<float>(ll)};
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        if (sb == 3 && !last) continue;
        const int64_t rowi = B.off[sb] + static_cast<int64_t>(ky) * B.Kx + kx;
        if (MODE == 0) {
          if (ok) A.w[rowi * L + p] = vb[sb];
        } else if (MODE == 1) {
          const float u = ok ? w[sb] + vb[sb] : 0.0f;
          const float wn = shrink<LCP>(u, thr * th[sb]);
          if (ok) A.w[rowi * L + p] = wn;
        } else {
          const float vv = ok ? vb[sb] : 0.0f;
          const float r2 = seg_sum(vv * vv, LCP);
          if (ok && lane == 0) A.theta[static_cast<int64_t>(c) * A.I + rowi] = thr / (sqrtf(r2) + thr);
        }
      }
      if (!last && ok)
        B.ll_out[(static_cast<int64_t>(ky) * B.Kx + kx) * L + p] = static_cast<float>(3.0 * ll);
    }
  };

  // two steps per iteration, the register sets alternating (no copies)
  for (int g = 0; g < nsteps; g += 2) {
    load_rows(g + 1, tb);
    load_emit(g + 1, wb, thb);
    step(g, ta, wa, tha);
    if (g + 1 < nsteps) {
      load_rows(g + 2, ta);
      load_emit(g + 2, wa, tha);
      step(g + 1, tb, wb, thb);
    }
  }
}

// Dirac basis: coefficient row = pixel; grid-stride over pixels, 4 in flight.
template <int MODE, int LCP>
__device__ __forceinline__ void dirac(const AnaArgs &A, const AnaBand &B, int wg) {
  const int L = A.L, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % LCP, grp = tid / LCP, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? c + lane * C : 0;
  constexpr int E = 4;
  // pixels of the rectangle [ky_begin, ky_end) x [kx_begin, kx_end), row-major
  const int rw = B.kx_end - B.kx_begin;
  const bool full = rw == B.in_nx;
  const int64_t npix = static_cast<int64_t>(B.ky_end - B.ky_begin) * rw;
  const int64_t pix_first = static_cast<int64_t>(B.ky_begin) * B.in_nx + B.kx_begin;
  const int64_t stride = static_cast<int64_t>(B.strips) * A.tkx1;  // strips = Dirac workgroups
  float thr = 0.0f;
  if (MODE == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (MODE == 2) thr = static_cast<float>(A.mu[c]);
  for (int64_t pix0 = static_cast<int64_t>(wg) * A.tkx1 + kq; pix0 - kq < npix; pix0 += E * stride) {
    float v[E], w[E], th[E];
    int64_t pixe[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t li = pix0 + e * stride;
      pixe[e] = full ? pix_first + li : pix_first + (li / rw) * B.in_nx + li % rw;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool ok = lv && pix0 + e * stride < npix;
      const int64_t pix = pixe[e];
      const int64_t i = B.off[0] + pix;
      v[e] = ok ? B.in[pix * L + chan] * (1.0f / 3.0f) : 0.0f;
      w[e] = (ok && MODE == 1) ? A.w[i * L + p] : 0.0f;
      th[e] = (ok && MODE == 1) ? A.theta[c * A.I + i] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool ok = lv && pix0 + e * stride < npix;
      const int64_t i = B.off[0] + pixe[e];
      if (MODE == 0) {
        if (ok) A.w[i * L + p] = v[e];
      } else if (MODE == 1) {
        const float wn = shrink<LCP>(ok ? w[e] + v[e] : 0.0f, thr * th[e]);
        if (ok) A.w[i * L + p] = wn;
      } else {
        const float r2 = seg_sum(v[e] * v[e], LCP);
        if (ok && lane == 0) A.theta[static_cast<int64_t>(c) * A.I + i] = thr / (sqrtf(r2) + thr);
      }
    }
  }
}

// FIRST: level 1 (reads the cube, also handles the Dirac basis); a separate
// instantiation so that its launches are timed and profiled on their own.
template <bool FIRST, int MODE, int LCP, bool DIRECT>
__global__ void __launch_bounds__(FHS_ANA_THREADS) kernel(AnaArgs A) {
  extern __shared__ float smem[];
  const int id = blockIdx.x;
  if (id < A.nbase_wg) {
#ifndef FHS_ANA_XCD
#define FHS_ANA_XCD 0
#endif
#if FHS_ANA_XCD == 1
    // tile t runs on XCD t % 8, its 8 bases in consecutive workgroups there
    const int x = id & 7, k = id >> 3;
    const int b = k & 7, tile = (k >> 3) * 8 + x;
#elif FHS_ANA_XCD == 2
    const int x = id & 7, k = id >> 3;
    const int b = k & 7, tile = x * A.tiles_per_xcd + (k >> 3);
#else
    const int b = id / (8 * A.tiles_per_xcd), tile = id - b * 8 * A.tiles_per_xcd;
#endif
    // static band indices, each band descriptor read into its own copy (a
    // dynamically indexed descriptor would be copied to scratch)
    switch (b) {
      case 0: { const AnaBand B = A.b[0]; if (DIRECT) basis_direct<2, MODE, LCP>(A, B, tile); else basis<2, MODE, LCP>(A, B, tile, smem); } break;
      case 1: { const AnaBand B = A.b[1]; if (DIRECT) basis_direct<4, MODE, LCP>(A, B, tile); else basis<4, MODE, LCP>(A, B, tile, smem); } break;
      case 2: { const AnaBand B = A.b[2]; if (DIRECT) basis_direct<6, MODE, LCP>(A, B, tile); else basis<6, MODE, LCP>(A, B, tile, smem); } break;
      case 3: { const AnaBand B = A.b[3]; if (DIRECT) basis_direct<8, MODE, LCP>(A, B, tile); else basis<8, MODE, LCP>(A, B, tile, smem); } break;
      case 4: { const AnaBand B = A.b[4]; if (DIRECT) basis_direct<10, MODE, LCP>(A, B, tile); else basis<10, MODE, LCP>(A, B, tile, smem); } break;
      case 5: { const AnaBand B = A.b[5]; if (DIRECT) basis_direct<12, MODE, LCP>(A, B, tile); else basis<12, MODE, LCP>(A, B, tile, smem); } break;
      case 6: { const AnaBand B = A.b[6]; if (DIRECT) basis_direct<14, MODE, LCP>(A, B, tile); else basis<14, MODE, LCP>(A, B, tile, smem); } break;
      default: { const AnaBand B = A.b[7]; if (DIRECT) basis_direct<16, MODE, LCP>(A, B, tile); else basis<16, MODE, LCP>(A, B, tile, smem); } break;
    }
  } else if (FIRST) {
    dirac<MODE, LCP>(A, A.b[kBases], id - A.nbase_wg);
  }
}

template <int MODE>
int launch_mode(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(a.nbase_wg + (first ? a.b[kBases].strips : 0))), block(nthreads);
#define FHS_ANA_CASE(LCP)                                                                      \
  case LCP:                                                                                    \
    if (a.direct) {                                                                            \
      if (first)                                                                               \
        hipLaunchKernelGGL((kernel<true, MODE, LCP, true>), grid, block, 0, s, a);             \
      else                                                                                     \
        hipLaunchKernelGGL((kernel<false, MODE, LCP, true>), grid, block, 0, s, a);            \
    } else {                                                                                   \
      if (first)                                                                               \
        hipLaunchKernelGGL((kernel<true, MODE, LCP, false>), grid, block, lds, s, a);          \
      else                                                                                     \
        hipLaunchKernelGGL((kernel<false, MODE, LCP, false>), grid, block, lds, s, a);         \
    }                                                                                          \
    break;
  switch (a.Lcp) {
    FHS_ANA_CASE(4)
    FHS_ANA_CASE(8)
    FHS_ANA_CASE(16)
    FHS_ANA_CASE(32)
    FHS_ANA_CASE(64)
    default:
      return fail(FHS_EUNSUPPORTED, "analysis: lanes per sub-cube must be 4..64");
  }
#undef FHS_ANA_CASE
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("analysis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

}  // namespace ana
}  // namespace fhs
