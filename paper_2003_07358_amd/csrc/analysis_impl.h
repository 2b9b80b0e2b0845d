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
// positions of every sub-cube, a segment of LCP lanes per sub-cube: padded
// to a power of two, or dense, see seg_map) and a run of
// coefficient rows of one basis at one level.  It streams input rows top to
// bottom: step g filters input rows 2g, 2g+1 (relative to the first needed row)
// horizontally into a per-thread FP64 register ring, and once the ring holds
// NTAP rows filters vertically to emit one coefficient row of the four bands.
//
// Memory pipeline: steps are grouped into phases of P steps.  Per phase, the
// 2P input row segments (and, for the dual update, the W and theta values of
// the P emitted rows) are copied HBM -> LDS by buffer loads whose destination
// is LDS, one phase ahead into a double buffer; one barrier per phase.  A
// staged row is laid out [sub-cube][column][lane slot] with LCP slots per
// column, so that the taps of a lane sit at compile-time offsets from one
// address (padding slots and columns outside the band read as zero); each
// lane's W and theta values are staged at its own thread index.  The results
// leave through range-checked buffer stores (out-of-range lanes are dropped),
// a fixed four per emitted row, so that the wait at a phase boundary can leave
// the previous phase's stores in flight.
//
// Launch order (a tuned launch parameter): workgroups are dealt to the 8 XCDs
// in turn, so each XCD walks its own run of consecutive tiles (horizontal and
// vertical neighbours share halo rows and columns through that XCD's L2).
// Basis-major: every tile of db8, then of db7, ... (the heaviest bases first,
// the light ones fill the tail).  Tile-major: the 8 bases of a tile back to
// back on one XCD, so that they read its input rows while they are in L2.
//
// Arithmetic: FP32 in / FP32 out, FP64 accumulation (detail coefficients are
// differences of large neighbouring values), unnormalised filters with the
// 1/3 applied to each emitted coefficient.  The mixed-precision form of the
// l21 update accumulates in FP32 instead (accumulator type T).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fhs_filters.h"
#include "fhs_internal.h"
#include "lds_stage.h"

namespace fhs {
namespace ana {

constexpr double kThird = 1.0 / 3.0;  // 1 / sqrt(9): nine bases
constexpr int kMaxPhase = 4;          // steps per LDS phase, upper bound (the launch picks P)
constexpr int kOob = static_cast<int>(0x80000000u);  // buffer offset past any range: loads 0, stores dropped

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

// Horizontal filters of one input row at one output column: lo = sum_m h[m]
// v_m and hi = sum_m g[m] v_m, g[m] = (-1)^m h[NTAP-1-m], where v_m = tap(m)
// is the input at column 2k+1-m.  The high-pass sign stays off the constants
// (even and odd terms are summed apart), so only the NTAP values h[m] are live.
template <int NTAP, typename T, typename F>
__device__ __forceinline__ void hfilt(F &&tap, T &lo, T &hi) {
  using TP = Taps<NTAP>;
  T sl = 0, se = 0, so = 0;
#pragma unroll
  for (int m = 0; m < NTAP; ++m) {
    const T v = static_cast<T>(tap(m));
    sl = fma(static_cast<T>(TP::hd[m]), v, sl);
    if (m & 1)
      so = fma(static_cast<T>(TP::hd[NTAP - 1 - m]), v, so);
    else
      se = fma(static_cast<T>(TP::hd[NTAP - 1 - m]), v, se);
  }
  lo = sl;
  hi = se - so;
}

// Vertical filters over the ring (ra(m), rb(m): the low and high horizontal
// outputs of the row that tap m multiplies): ll, lh through h, hl, hh through g.
template <int NTAP, typename T, typename FA, typename FB>
__device__ __forceinline__ void vfilt(FA &&ra, FB &&rb, T &ll, T &lh, T &hl, T &hh) {
  using TP = Taps<NTAP>;
  T sll = 0, slh = 0, ae = 0, ao = 0, be = 0, bo = 0;
#pragma unroll
  for (int m = 0; m < NTAP; ++m) {
    const T a = ra(m), b = rb(m);
    sll = fma(static_cast<T>(TP::hd[m]), a, sll);
    slh = fma(static_cast<T>(TP::hd[m]), b, slh);
    if (m & 1) {
      ao = fma(static_cast<T>(TP::hd[NTAP - 1 - m]), a, ao);
      bo = fma(static_cast<T>(TP::hd[NTAP - 1 - m]), b, bo);
    } else {
      ae = fma(static_cast<T>(TP::hd[NTAP - 1 - m]), a, ae);
      be = fma(static_cast<T>(TP::hd[NTAP - 1 - m]), b, be);
    }
  }
  ll = sll;
  lh = slh;
  hl = ae - ao;
  hh = be - bo;
}

__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void st_f32(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}
// Raw buffer over [base, base + bytes): offsets at or past `bytes` read zero
// and drop their stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0), static_cast<int>(bytes),
                                           0x00020000);
}

// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>), in order.
template <int I, int N>
struct Unroll {
  template <typename F>
  __device__ __forceinline__ static void run(F &&f) {
    f(std::integral_constant<int, I>{});
    Unroll<I + 1, N>::run(f);
  }
};
template <int N>
struct Unroll<N, N> {
  template <typename F>
  __device__ __forceinline__ static void run(F &&) {}
};
template <int N, typename F>
__device__ __forceinline__ void unroll_steps(F &&f) {
  Unroll<0, N>::run(f);
}

// Workgroup barrier without a memory fence (the copies are waited for by
// count before it; LDS accesses are not moved across it).
__device__ __forceinline__ void barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Waits until at most n (0, 4, 8 or 16) of this wave's vector-memory
// operations are outstanding.  They complete in issue order, so the n most
// recent may stay in flight.
__device__ __forceinline__ void wait_vm_but(int n) {
  if (n == 4)
    asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  else if (n == 8)
    asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
  else if (n == 16)
    asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
  else
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Mode 3: bit sy set when facet (sy, sx) of sub-cube c is selected (at most
// 64 facet rows).
__device__ __forceinline__ uint64_t sel_bits(const AnaArgs &A, int c, int sx) {
  uint64_t m = 0;
  for (int sy = 0; sy < A.qy; ++sy)
    if (A.sel[(c * A.qy + sy) * A.qx + sx] != 0) m |= uint64_t{1} << sy;
  return m;
}

template <int NTAP, int MODE, int LCP, typename T>
__device__ __forceinline__ void basis(const AnaArgs &A, const AnaBand &B, int tile, float *smem) {
  constexpr int H = NTAP / 2;
  if (tile >= B.strips * B.yblocks) return;
  const int L = A.L, C = A.C, Lc = A.Lc, P = A.P;
  const int tid = threadIdx.x;
  int lane, grp;
  bool idle;
  seg_map(tid, LCP, lane, grp, idle);
  const int TKX = A.tkx1;
  // (segments past the tile's TKX columns, possible with dense widths, work
  // on column 0 and store nothing)
  const int c = grp % C, kq = grp / C < TKX ? grp / C : 0;
  const int p = c * Lc + lane;
  const int strip = tile % B.strips, yb = tile / B.strips;
  const int kx0 = B.kx_begin + strip * TKX, ky0 = B.ky_begin + yb * A.tky;
  const int ky1 = min(ky0 + A.tky, B.ky_end);
  const int nkx = min(TKX, B.kx_end - kx0);     // coefficient columns of the tile
  const bool ok = !idle && lane < Lc && grp / C < nkx;
  const int NC = 2 * TKX + NTAP - 2;            // input columns of a staged row
  const int NCP = NC + (C > 1 ? 1 : 0);         // columns per sub-cube block (one pad column spreads the
                                                // sub-cube blocks over the LDS banks)
  // 16-byte copies when the channels of a column segment are contiguous and
  // 16-byte aligned, else 4-byte copies; a chunk is one copy instruction
  const bool v4 = A.vec4 && (C == 1 || !B.in_natural);
  const int cw = v4 ? 256 : 64;                 // words per chunk
  const int nchunk = (C * NCP * LCP + cw - 1) / cw;
  const int ROW = A.lds_row;
  const int col0 = 2 * kx0 + 2 - NTAP;          // first input column
  const int ystart = 2 * ky0 + 2 - NTAP;
  const int nsteps = (ky1 - ky0) + H - 1;
  const int nph = (nsteps + P - 1) / P;
  const uint32_t row_bytes = static_cast<uint32_t>(B.in_nx) * L * 4;
  const bool last = B.ll_out == nullptr;
  const uint32_t run_bytes = static_cast<uint32_t>(nkx * L * 4);  // one coefficient row run of the tile
  const uint64_t band_row = static_cast<uint64_t>(B.Kx) * L * 4;  // bytes per coefficient row of a band
  float thr = 0.0f;
  if (MODE == 1 || MODE == 3) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (MODE == 2) thr = static_cast<float>(A.mu[c]);
  // a frozen sub-cube keeps its old W (mode 1) or theta (mode 2)
  const bool act = A.active == nullptr || A.active[c] != 0;
  const int wv = wave_id(), nwv = full_wave_count(), ln = tid & 63;

  // byte addresses of the tile's first column in coefficient row 0 of each
  // band (W) and of the low-low output; theta row offsets of the bands
  const char *wbase[4];
  int32_t tbase[4];
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    // (explicit select: a dynamic index into the band descriptor would copy it to scratch)
    const int64_t boff = sb == 0 ? B.off[0] : sb == 1 ? B.off[1] : sb == 2 ? B.off[2] : B.off[3];
    wbase[sb] = reinterpret_cast<const char *>(A.w + (boff + kx0) * L);
    tbase[sb] = static_cast<int32_t>(boff * 4);
  }
  const char *llbase = reinterpret_cast<const char *>(B.ll_out + static_cast<int64_t>(kx0) * L);

  // buffer offsets of this lane: its word in a coefficient row run of the
  // tile (W, low-low output) and its theta word (sub-cube c, column kx)
  const int wl = kq * L + p;
  const int vo = ok ? wl * 4 : kOob;
  const int vth = ok ? static_cast<int>((static_cast<int64_t>(c) * A.I + kx0 + kq) * 4) : kOob;
  const int vth0 = lane == 0 ? vth : kOob;
  // mode 3: bit sy of this lane's mask = facet (sy, owner column of its
  // coefficient column) is selected
  const uint64_t selbits = MODE == 3 && ok ? sel_bits(A, c, A.own[B.own_c + kx0 + kq]) : 0;
  // theta copy: word i = 64 j + ln of a segment -> (sub-cube i / TKX, column i % TKX)
  int th_voff[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = 64 * j + ln, cc = i / TKX, kk = i - cc * TKX;
    th_voff[j] = (cc < C && kk < nkx) ? static_cast<int>((static_cast<int64_t>(cc) * A.I + kx0 + kk) * 4) : kOob;
  }
  const int nth_chunks = (C * TKX + 63) >> 6;

  // copy table (all waves build it): for chunk i of a staged row, lane ln's
  // byte offset in the input row, or out of range
  int *tab = reinterpret_cast<int *>(smem + A.lds_tab);
  for (int e = tid; e < nchunk * 64; e += blockDim.x) {
    const int s0 = (e >> 6) * cw + (e & 63) * (cw >> 6);  // first slot of the lane's copy
    const int ls = s0 % LCP, q = s0 / LCP, cc = q / NCP, col = q - cc * NCP, gc = col0 + col;
    int off = kOob;
    if (cc < C && col < NC && ls < Lc && gc >= 0 && gc < B.in_nx)
      off = (gc * L + (B.in_natural ? cc + ls * C : cc * Lc + ls)) * 4;
    tab[e] = off;
  }
  __syncthreads();
  const int *tabl = tab + ln;

  // one phase of copies: the 2P input rows (one wave each), and for the dual
  // update the W run and the theta values of each row emitted in the phase
  // (one wave per band and row), spread over the full waves
  const int ntask = 2 * P + (MODE == 1 || MODE == 3 ? 8 * P : 0);
  auto issue_phase = [&](int ph) __attribute__((always_inline)) {
    float *buf = smem + (ph & 1) * A.lds_buf;
    for (int t = wv; t < ntask && wv < nwv; t += nwv) {
      if (t < 2 * P) {
        const int y = ystart + 2 * P * ph + t;
        const bool yv = y >= 0 && y < B.in_ny;
        const fhs_int32x4 rs =
            buffer_rsrc(reinterpret_cast<const char *>(B.in) + (yv ? static_cast<uint64_t>(y) * row_bytes : 0),
                        yv ? row_bytes : 0u);
        float *dst = buf + t * ROW;
        if (v4) {
          for (int i = 0; i < nchunk; ++i) fhs_raw_buffer_load_lds(rs, lds_ptr(dst + 256 * i), 16, tabl[64 * i], 0, 0, 0);
        } else {
          for (int i = 0; i < nchunk; ++i) fhs_raw_buffer_load_lds(rs, lds_ptr(dst + 64 * i), 4, tabl[64 * i], 0, 0, 0);
        }
      } else {
        const int u = t - 2 * P, k = u >> 3, sb = u & 3;
        const int g = P * ph + k;
        if (g >= nsteps || g < H - 1 || (sb == 3 && !last)) continue;
        const int ky = ky0 + g - (H - 1);
        const int64_t boff = sb == 0 ? B.off[0] : sb == 1 ? B.off[1] : sb == 2 ? B.off[2] : B.off[3];
        if ((u & 4) == 0) {
          // W run of the row: nkx L contiguous floats
          const fhs_int32x4 wr = buffer_rsrc(reinterpret_cast<const char *>(A.w + (boff + kx0) * L) +
                                                 static_cast<uint64_t>(ky) * band_row,
                                             run_bytes);
          float *dst = buf + A.lds_wv + (4 * k + sb) * kAnaLaneSeg;
          if (A.vec4)
            for (int j = 0; j < kAnaLaneSeg; j += 256) fhs_raw_buffer_load_lds(wr, lds_ptr(dst + j), 16, (j + 4 * ln) * 4, 0, 0, 0);
          else
            for (int j = 0; j < kAnaLaneSeg; j += 64) fhs_raw_buffer_load_lds(wr, lds_ptr(dst + j), 4, (j + ln) * 4, 0, 0, 0);
        } else {
          // theta of the row for every sub-cube: a gather
          const fhs_int32x4 tr = buffer_rsrc(A.theta, static_cast<unsigned>(A.theta_bytes));
          float *dst = buf + A.lds_th + (4 * k + sb) * kAnaThSeg;
          const int so = static_cast<int>((boff + static_cast<int64_t>(ky) * B.Kx) * 4);
          fhs_raw_buffer_load_lds(tr, lds_ptr(dst), 4, th_voff[0], so, 0, 0);
          if (nth_chunks > 1) fhs_raw_buffer_load_lds(tr, lds_ptr(dst + 64), 4, th_voff[1], so, 0, 0);
        }
      }
    }
  };

  // ring of horizontal outputs: slot i % NTAP holds input row i (relative to
  // the first needed row); the loop below is unrolled over H steps, so that
  // every slot index is a compile-time constant and no entry moves
  T rl[NTAP], rh[NTAP];
#pragma unroll
  for (int m = 0; m < NTAP; ++m) rl[m] = rh[m] = 0;
  // LDS word of tap NTAP-1 (the lowest column) of this lane in a staged row
  const int lb = (c * NCP + 2 * kq) * LCP + lane;
  const int tl = c * TKX + kq;  // lane's word in a theta segment

  issue_phase(0);
  int ph = 0, k = 0;
  // step g at ring rotation S (= g mod H when the loop is unrolled over H
  // steps, else H-1 after a shift of the ring by two)
  auto phase_top = [&]() __attribute__((always_inline)) {
    if (k == 0) {
      // the phase's copies were issued before the previous phase's 4P
      // stores, the only later vector-memory operations of this wave; the
      // barrier itself waits for nothing
      if (ph == 0)
        wait_vm_but(0);
      else
        wait_vm_but(4 * P);
      barrier();
      if (ph + 1 < nph) issue_phase(ph + 1);
    }
  };
  auto step = [&](auto S, int g) __attribute__((always_inline)) {
    constexpr int s = decltype(S)::value;
    const float *buf = smem + (ph & 1) * A.lds_buf;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const float *rp = buf + (2 * k + r) * ROW + lb;
      hfilt<NTAP, T>([&](int m) { return rp[(NTAP - 1 - m) * LCP]; }, rl[2 * s + r], rh[2 * s + r]);
    }
    if (g >= H - 1) {
      // tap m multiplies input row 2g+1-m, slot (2s+1-m) mod NTAP
      T ll, lh, hl, hh;
      vfilt<NTAP, T>([&](int m) { return rl[(2 * s + 1 - m + NTAP) % NTAP]; },
                  [&](int m) { return rh[(2 * s + 1 - m + NTAP) % NTAP]; }, ll, lh, hl, hh);
      const int ky = ky0 + g - (H - 1);
      const uint64_t rb = static_cast<uint64_t>(ky) * band_row;
      const T third = static_cast<T>(kThird);
      const float vb[4] = {static_cast<float>(lh * third), static_cast<float>(hl * third),
                           static_cast<float>(hh * third), static_cast<float>(ll * third)};
      const float *wsg = buf + A.lds_wv + 4 * k * kAnaLaneSeg + wl;
      const float *tsg = buf + A.lds_th + 4 * k * kAnaThSeg + tl;
      // exactly four stores per emitted row (the phase wait counts them)
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        if (sb == 3 && !last) continue;
        if (MODE == 0) {
          st_f32(vb[sb], rsrc(wbase[sb] + rb, run_bytes), vo, 0);
        } else if (MODE == 1 || MODE == 3) {
          const float wold = wsg[sb * kAnaLaneSeg], th = tsg[sb * kAnaThSeg];
          const float u = lane < Lc ? wold + vb[sb] : 0.0f;
          const float wn = shrink<LCP>(u, thr * th);
          const bool upd = MODE == 3 ? ((selbits >> A.own[B.own_r + ky]) & 1) != 0 : act;
          st_f32(upd ? wn : wold, rsrc(wbase[sb] + rb, run_bytes), vo, 0);
        } else {
          const float r2 = seg_sum(vb[sb] * vb[sb], LCP);
          st_f32(thr / (sqrtf(r2) + thr), rsrc(A.theta, static_cast<uint32_t>(A.theta_bytes)), act ? vth0 : kOob,
                 tbase[sb] + ky * B.Kx * 4);
        }
      }
      if (!last) st_f32(static_cast<float>(ll), rsrc(llbase + rb, run_bytes), vo, 0);
    } else {
      // (steps that fill the ring issue four dropped stores, so that every
      // step issues exactly four; distinct, non-adjacent offsets keep the
      // compiler from merging or eliminating them)
      const __amdgpu_buffer_rsrc_t none = rsrc(A.w, 0u);
#pragma unroll
      for (int i = 0; i < 4; ++i) st_f32(0.0f, none, kOob + 1024 * i, 0);
    }
    if (++k == P) {
      k = 0;
      ++ph;
    }
  };
  // one copy of the phase code, H copies of the step body (one per ring
  // rotation, selected by g mod H)
  for (int g = 0, s = 0; g < nsteps; ++g) {
    phase_top();
    unroll_steps<H>([&](auto S) __attribute__((always_inline)) {
      if (s == decltype(S)::value) step(S, g);
    });
    s = s + 1 == H ? 0 : s + 1;
  }
  drain_loads();  // no LDS copy may land after the workgroup ends
}

// The same computation without LDS: every lane loads its own filter taps and
// W / theta straight from HBM (through the caches) one step ahead into
// registers, with range-checked buffer loads (out-of-range columns and rows
// read as zero).  No barriers; the compiler's wait counts track each load, so
// stores never stall a step.

template <int NTAP, int MODE, int LCP, typename T>
__device__ __forceinline__ void basis_direct(const AnaArgs &A, const AnaBand &B, int tile) {
  constexpr int H = NTAP / 2;
  if (tile >= B.strips * B.yblocks) return;
  const int L = A.L, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  int lane, grp;
  bool idle;
  seg_map(tid, LCP, lane, grp, idle);
  const int TKX = A.tkx1;
  const int c = grp % C, kq = grp / C < TKX ? grp / C : 0;
  const bool lv = !idle && lane < Lc && grp / C < TKX;
  const int p = c * Lc + lane;
  const int chan = lv ? (B.in_natural ? c + lane * C : p) : 0;
  const int strip = tile % B.strips, yb = tile / B.strips;
  const int kx0 = B.kx_begin + strip * TKX, ky0 = B.ky_begin + yb * A.tky;
  const int ky1 = min(ky0 + A.tky, B.ky_end);
  const int kx = kx0 + kq;
  const bool ok = lv && kx < B.kx_end;
  const int ystart = 2 * ky0 + 2 - NTAP;
  const int nsteps = (ky1 - ky0) + H - 1;
  const int64_t rowlen = static_cast<int64_t>(B.in_nx) * L;
  float thr = 0.0f;
  if (MODE == 1 || MODE == 3) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (MODE == 2) thr = static_cast<float>(A.mu[c]);
  const bool act = A.active == nullptr || A.active[c] != 0;  // frozen sub-cubes keep W / theta
  const uint64_t selbits = MODE == 3 && ok ? sel_bits(A, c, A.own[B.own_c + kx]) : 0;
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
      if (MODE == 1 || MODE == 3) {
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

  T rl[NTAP], rh[NTAP];
#pragma unroll
  for (int m = 0; m < NTAP; ++m) rl[m] = rh[m] = 0;
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
    for (int r = 0; r < 2; ++r) hfilt<NTAP, T>([&](int m) { return t[r][m]; }, rl[NTAP - 2 + r], rh[NTAP - 2 + r]);
    if (g >= H - 1) {
      T ll, lh, hl, hh;
      vfilt<NTAP, T>([&](int m) { return rl[NTAP - 1 - m]; }, [&](int m) { return rh[NTAP - 1 - m]; }, ll, lh, hl,
                     hh);
      const int ky = ky0 + g - (H - 1);
      const T third = static_cast<T>(kThird);
      const float vb[4] = {static_cast<float>(lh * third), static_cast<float>(hl * third),
                           static_cast<float>(hh * third), static_cast<float>(ll * third)};
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        if (sb == 3 && !last) continue;
        const int64_t rowi = B.off[sb] + static_cast<int64_t>(ky) * B.Kx + kx;
        if (MODE == 0) {
          if (ok) A.w[rowi * L + p] = vb[sb];
        } else if (MODE == 1 || MODE == 3) {
          // (lanes past Lc load channel 0: kept out of the norm)
          const float wn = shrink<LCP>(lv ? w[sb] + vb[sb] : 0.0f, thr * th[sb]);
          const bool upd = MODE == 3 ? ((selbits >> A.own[B.own_r + ky]) & 1) != 0 : act;
          if (ok && upd) A.w[rowi * L + p] = wn;
        } else {
          const float vv = lv ? vb[sb] : 0.0f;
          const float r2 = seg_sum(vv * vv, LCP);
          if (ok && act && lane == 0) A.theta[static_cast<int64_t>(c) * A.I + rowi] = thr / (sqrtf(r2) + thr);
        }
      }
      if (!last && ok) B.ll_out[(static_cast<int64_t>(ky) * B.Kx + kx) * L + p] = static_cast<float>(ll);
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

// Dirac basis (Sec. 2.3.1: the identity as ninth basis, divided by 3):
// coefficient row = pixel, an elementwise pass.  Its own launch without LDS
// (so that many workgroups stay resident), grid-stride over the pixels of the
// rectangle [ky_begin, ky_end) x [kx_begin, kx_end), E pixels per thread in
// flight and the next E loaded before the current ones are updated.
template <int MODE, int LCP>
__global__ void __launch_bounds__(kDiracThreads) dirac_kernel(AnaArgs A) {
  constexpr int E = kDiracE;
  const AnaBand &B = A.b[kBases];
  const int L = A.L, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  int lane, grp;
  bool idle;
  seg_map(tid, LCP, lane, grp, idle);
  const int c = grp % C, kq = grp / C;
  // pixels per workgroup and pass
  const int ppw = dense_width(LCP) ? dense_segments(blockDim.x, LCP) / C : blockDim.x / (C * LCP);
  const bool lv = !idle && lane < Lc && kq < ppw;
  const int p = c * Lc + lane;
  const int chan = lv ? (B.in_natural ? c + lane * C : p) : 0;
  const int rw = B.kx_end - B.kx_begin;
  const bool full = rw == B.in_nx;
  const int64_t npix = static_cast<int64_t>(B.ky_end - B.ky_begin) * rw;
  const int64_t pix_first = static_cast<int64_t>(B.ky_begin) * B.in_nx + B.kx_begin;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * ppw;
  float thr = 0.0f;
  if (MODE == 1 || MODE == 3) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (MODE == 2) thr = static_cast<float>(A.mu[c]);
  const bool act = A.active == nullptr || A.active[c] != 0;  // frozen sub-cubes keep W / theta
  auto pixel = [&](int64_t li) { return full ? pix_first + li : pix_first + (li / rw) * B.in_nx + li % rw; };
  auto load = [&](int64_t l0, float (&v)[E], float (&w)[E], float (&th)[E]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t li = l0 + e * stride;
      const bool ok = lv && li < npix;
      const int64_t pix = ok ? pixel(li) : 0;
      const int64_t i = B.off[0] + pix;
      v[e] = ok ? B.in[pix * L + chan] : 0.0f;
      w[e] = (ok && (MODE == 1 || MODE == 3)) ? A.w[i * L + p] : 0.0f;
      th[e] = (ok && (MODE == 1 || MODE == 3)) ? A.theta[c * A.I + i] : 0.0f;
    }
  };
  const int64_t first = static_cast<int64_t>(blockIdx.x) * ppw + kq;
  float v[E], w[E], th[E];
  load(first, v, w, th);
  for (int64_t l0 = first; l0 - kq < npix; l0 += E * stride) {
    float vn[E], wn[E], thn[E];
    load(l0 + E * stride, vn, wn, thn);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t li = l0 + e * stride;
      const bool ok = lv && li < npix;
      const int64_t i = B.off[0] + (ok ? pixel(li) : 0);
      const float x3 = v[e] * (1.0f / 3.0f);
      if (MODE == 0) {
        if (ok) A.w[i * L + p] = x3;
      } else if (MODE == 1 || MODE == 3) {
        const float nw = l21_row_update(w[e], v[e], thr * th[e], LCP);
        bool upd = act;
        if (MODE == 3 && ok) {
          // the pixel's tile is the owner facet of its Dirac row
          const int64_t pix = pixel(li), yy = pix / B.in_nx;
          const int sy = A.own[B.own_r + yy], sx = A.own[B.own_c + (pix - yy * B.in_nx)];
          upd = A.sel[(c * A.qy + sy) * A.qx + sx] != 0;
        }
        if (ok && upd) A.w[i * L + p] = nw;
      } else {
        const float r2 = seg_sum(x3 * x3, LCP);
        if (ok && act && lane == 0) A.theta[static_cast<int64_t>(c) * A.I + i] = thr / (sqrtf(r2) + thr);
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = vn[e];
      w[e] = wn[e];
      th[e] = thn[e];
    }
  }
}

// FIRST: level 1 (reads the cube); a separate instantiation so that its
// launches are profiled on their own.
template <bool FIRST, int MODE, int LCP, bool DIRECT, typename T>
__device__ __forceinline__ void kernel_body(const AnaArgs &A, float *smem) {
  const int id = blockIdx.x;
  if (id < A.nbase_wg) {
    int b, tile;
    if (A.tile_major) {
      // XCD x = id mod 8 takes its k-th workgroup: the 8 bases of its tile k / 8
      const int x = id & 7, k = id >> 3;
      b = 7 - (k & 7);
      tile = x * A.tiles_per_xcd + (k >> 3);
    } else {
      const int per_basis = 8 * A.tiles_per_xcd, r = id - (id / per_basis) * per_basis;
      b = 7 - id / per_basis;
      tile = (r & 7) * A.tiles_per_xcd + (r >> 3);
    }
    // static band indices, each band descriptor read into its own copy (a
    // dynamically indexed descriptor would be copied to scratch)
    switch (b) {
      case 0: { const AnaBand B = A.b[0]; if (DIRECT) basis_direct<2, MODE, LCP, T>(A, B, tile); else basis<2, MODE, LCP, T>(A, B, tile, smem); } break;
      case 1: { const AnaBand B = A.b[1]; if (DIRECT) basis_direct<4, MODE, LCP, T>(A, B, tile); else basis<4, MODE, LCP, T>(A, B, tile, smem); } break;
      case 2: { const AnaBand B = A.b[2]; if (DIRECT) basis_direct<6, MODE, LCP, T>(A, B, tile); else basis<6, MODE, LCP, T>(A, B, tile, smem); } break;
      case 3: { const AnaBand B = A.b[3]; if (DIRECT) basis_direct<8, MODE, LCP, T>(A, B, tile); else basis<8, MODE, LCP, T>(A, B, tile, smem); } break;
      case 4: { const AnaBand B = A.b[4]; if (DIRECT) basis_direct<10, MODE, LCP, T>(A, B, tile); else basis<10, MODE, LCP, T>(A, B, tile, smem); } break;
      case 5: { const AnaBand B = A.b[5]; if (DIRECT) basis_direct<12, MODE, LCP, T>(A, B, tile); else basis<12, MODE, LCP, T>(A, B, tile, smem); } break;
      case 6: { const AnaBand B = A.b[6]; if (DIRECT) basis_direct<14, MODE, LCP, T>(A, B, tile); else basis<14, MODE, LCP, T>(A, B, tile, smem); } break;
      default: { const AnaBand B = A.b[7]; if (DIRECT) basis_direct<16, MODE, LCP, T>(A, B, tile); else basis<16, MODE, LCP, T>(A, B, tile, smem); } break;
    }
  }
}

#ifndef FHS_ANA_WAVES_PER_EU
#define FHS_ANA_WAVES_PER_EU 4  // register budget of the staged kernel: 128 VGPRs (two 512-thread workgroups per CU)
#endif
// (T: FP64 accumulation, or FP32 in the mixed-precision form)
template <bool FIRST, int MODE, int LCP, typename T>
__global__ void __launch_bounds__(FHS_ANA_THREADS) __attribute__((amdgpu_waves_per_eu(FHS_ANA_WAVES_PER_EU)))
kernel(AnaArgs A) {
  extern __shared__ float smem[];
  kernel_body<FIRST, MODE, LCP, false, T>(A, smem);
}

// the LDS-free variant keeps its taps in registers (no waves-per-SIMD target)
template <bool FIRST, int MODE, int LCP, typename T>
__global__ void __launch_bounds__(FHS_ANA_THREADS) kernel_direct(AnaArgs A) {
  kernel_body<FIRST, MODE, LCP, true, T>(A, nullptr);
}

template <int MODE, typename T = double>
int launch_mode(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(a.nbase_wg)), block(nthreads);
  const dim3 dgrid(static_cast<unsigned>(first ? a.b[kBases].strips : 0)), dblock(kDiracThreads);
// (the Dirac band always runs on padded segments, DLCP: the level-1
// synthesis, which fuses its update in the batched step, uses those too)
#define FHS_ANA_CASE2(LCP, DLCP)                                                               \
  case LCP:                                                                                    \
    if (dgrid.x > 0) hipLaunchKernelGGL((dirac_kernel<MODE, DLCP>), dgrid, dblock, 0, s, a);   \
    if (grid.x == 0) break;                                                                    \
    if (a.direct) {                                                                            \
      if (first)                                                                               \
        hipLaunchKernelGGL((kernel_direct<true, MODE, LCP, T>), grid, block, 0, s, a);          \
      else                                                                                     \
        hipLaunchKernelGGL((kernel_direct<false, MODE, LCP, T>), grid, block, 0, s, a);         \
    } else {                                                                                   \
      if (first)                                                                               \
        hipLaunchKernelGGL((kernel<true, MODE, LCP, T>), grid, block, lds, s, a);               \
      else                                                                                     \
        hipLaunchKernelGGL((kernel<false, MODE, LCP, T>), grid, block, lds, s, a);              \
    }                                                                                          \
    break;
#define FHS_ANA_CASE(LCP) FHS_ANA_CASE2(LCP, LCP)
  switch (a.Lcp) {
    FHS_ANA_CASE(4)
    FHS_ANA_CASE2(6, 8)
    FHS_ANA_CASE(8)
    FHS_ANA_CASE2(10, 16)
    FHS_ANA_CASE2(12, 16)
    FHS_ANA_CASE(16)
    FHS_ANA_CASE2(18, 32)
    FHS_ANA_CASE2(20, 32)
    FHS_ANA_CASE(32)
    FHS_ANA_CASE(64)
    default:
      return fail(FHS_EUNSUPPORTED, "analysis: unsupported lanes per sub-cube");
  }
#undef FHS_ANA_CASE
#undef FHS_ANA_CASE2
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("analysis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

}  // namespace ana
}  // namespace fhs
