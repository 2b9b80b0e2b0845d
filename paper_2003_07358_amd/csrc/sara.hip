// SARA analysis / synthesis kernels for gfx950 (Sec. 2.3.1, Alg. 2 steps
// alg:step:dual_sparsity and alg:step:end_facet-l21).
//
// Transform: zero-extended expansive separable DWT with the causal index
// convention a[k] = sum_m h[m] x[2k+1-m] (k < floor((n+L-1)/2)), applied along
// rows then columns, recursing on the low-low band; every stored coefficient
// is divided by 3 (nine bases).  The faceted transform of Sec. 2.4.2 equals
// this global one, so the kernels tile the global transform.
//
// Layout: bands are [rows][cols][L] with the L channel positions contiguous.
// A workgroup owns a strip of coefficient columns and a run of coefficient
// rows; thread (group, lane) handles one channel position of one column, the
// channels of a sub-cube being Lcp (power of two) consecutive lanes so that
// the l21 row norm across channels is a butterfly inside the wavefront.
// Input rows are staged through LDS (coalesced: a strip row is contiguous in
// HBM); the vertical filter keeps a per-thread ring of horizontally filtered
// rows in registers, indexed at compile time by unrolling over one filter
// length of rows.
#include <hip/hip_runtime.h>

#include "fhs_filters.h"
#include "fhs_internal.h"

#ifndef FHS_FINAL_SPLIT
#define FHS_FINAL_SPLIT 4
#endif
#ifndef FHS_FINAL_WPE
#define FHS_FINAL_WPE 2
#endif

namespace fhs {

__device__ __forceinline__ float seg_sum(float v, int lcp) {
  for (int o = 1; o < lcp; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Writes / updates one coefficient (value already divided by 3) at row i.
__device__ __forceinline__ void emit_coef(const AnaArgs &A, int64_t i, bool ok, int p, int c, int lane,
                                          float v, float thr) {
  if (A.mode == 0) {
    if (ok) A.w[i * A.L + p] = v;
  } else if (A.mode == 1) {
    // u = W_i + [Psi^dagger x]_i ; W_i <- u min(1, thr theta_i / ||u||)
    const float u = ok ? A.w[i * A.L + p] + v : 0.0f;
    const float r2 = seg_sum(u * u, A.Lcp);
    const float th = ok ? A.theta[c * A.I + i] : 0.0f;
    const float s = r2 > 0.0f ? fminf(1.0f, thr * th / sqrtf(r2)) : 0.0f;
    if (ok) A.w[i * A.L + p] = u * s;
  } else {
    // theta_i = upsilon / (||[Psi^dagger x]_i|| + upsilon)
    const float vv = ok ? v : 0.0f;
    const float r2 = seg_sum(vv * vv, A.Lcp);
    if (ok && lane == 0) A.theta[c * A.I + i] = thr / (sqrtf(r2) + thr);
  }
}

template <int NTAP, int E>
__device__ __forceinline__ void ana_basis(const AnaArgs &A, const AnaBand &B, int wg, float *buf) {
  using T = Taps<NTAP>;
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid % Lcp, grp = tid / Lcp, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? (B.in_natural ? c + lane * C : p) : 0;
  const int TKX = E * A.tkx1;
  const int strip = wg % B.strips, yb = wg / B.strips;
  const int kx0 = strip * TKX, ky0 = yb * A.tky;
  const int ky1 = min(ky0 + A.tky, B.Ky);
  const int segn = (2 * TKX + NTAP - 2) * L;
  const int64_t rowlen = static_cast<int64_t>(B.in_nx) * L;
  const int64_t seg0 = static_cast<int64_t>(2 * kx0 + 2 - NTAP) * L;
  const int nrows = 2 * (ky1 - ky0) + NTAP - 2;
  const int ystart = 2 * ky0 + 2 - NTAP;
  const float third = 1.0f / 3.0f;
  float thr = 0.0f;
  if (A.mode == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (A.mode == 2) thr = static_cast<float>(A.mu[c]);

  float rl[E][NTAP], rh[E][NTAP];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int m = 0; m < NTAP; ++m) rl[e][m] = rh[e][m] = 0.0f;

  for (int r0 = 0; r0 < nrows; r0 += NTAP) {
#pragma unroll
    for (int u = 0; u < NTAP; ++u) {
      const int r = r0 + u;
      if (r < nrows) {
        const int y = ystart + r;
        __syncthreads();
        if (y >= 0 && y < B.in_ny) {
          const float *rowp = B.in + static_cast<int64_t>(y) * rowlen;
          for (int i = tid; i < segn; i += nth) {
            const int64_t gi = seg0 + i;
            buf[i] = (gi >= 0 && gi < rowlen) ? rowp[gi] : 0.0f;
          }
        } else {
          for (int i = tid; i < segn; i += nth) buf[i] = 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float *bp = buf + (2 * (kq + e * A.tkx1) + NTAP - 1) * L + chan;
          float sl = 0.0f, sh = 0.0f;
#pragma unroll
          for (int m = 0; m < NTAP; ++m) {
            const float v = bp[-m * L];
            sl = fmaf(T::h[m], v, sl);
            sh = fmaf(T::g[m], v, sh);
          }
          rl[e][u] = sl;
          rh[e][u] = sh;
        }
        if ((u & 1) && r >= NTAP - 1) {
          const int ky = ky0 + ((r - (NTAP - 1)) >> 1);
#pragma unroll
          for (int e = 0; e < E; ++e) {
            float ll = 0.0f, lh = 0.0f, hl = 0.0f, hh = 0.0f;
#pragma unroll
            for (int m = 0; m < NTAP; ++m) {
              const int s = (u - m + NTAP) % NTAP;
              ll = fmaf(T::h[m], rl[e][s], ll);
              lh = fmaf(T::h[m], rh[e][s], lh);
              hl = fmaf(T::g[m], rl[e][s], hl);
              hh = fmaf(T::g[m], rh[e][s], hh);
            }
            const int kx = kx0 + kq + e * A.tkx1;
            const bool ok = lv && kx < B.Kx;
            const int64_t pos = static_cast<int64_t>(ky) * B.Kx + kx;
            emit_coef(A, B.off[0] + pos, ok, p, c, lane, lh * third, thr);
            emit_coef(A, B.off[1] + pos, ok, p, c, lane, hl * third, thr);
            emit_coef(A, B.off[2] + pos, ok, p, c, lane, hh * third, thr);
            if (B.ll_out) {
              if (ok) B.ll_out[pos * L + p] = ll;
            } else {
              emit_coef(A, B.off[3] + pos, ok, p, c, lane, ll * third, thr);
            }
          }
        }
      }
    }
  }
}

// Dirac basis: coefficient row = pixel.
template <int E>
__device__ __forceinline__ void ana_dirac(const AnaArgs &A, const AnaBand &B, int wg) {
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % Lcp, grp = tid / Lcp, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int chan = lv ? c + lane * C : 0;
  const int TKX = E * A.tkx1;
  const int64_t npix = static_cast<int64_t>(B.in_ny) * B.in_nx;
  float thr = 0.0f;
  if (A.mode == 1) thr = static_cast<float>(A.mu[c] * A.inv_kappa);
  if (A.mode == 2) thr = static_cast<float>(A.mu[c]);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t pix = static_cast<int64_t>(wg) * TKX + kq + e * A.tkx1;
    const bool ok = lv && pix < npix;
    const float v = ok ? B.in[pix * L + chan] * (1.0f / 3.0f) : 0.0f;
    emit_coef(A, B.off[0] + pix, ok, p, c, lane, v, thr);
  }
}

// FIRST: level 1 (reads the cube, also updates the Dirac basis); a separate
// instantiation so that its launches are timed and profiled on their own.
template <int E, bool FIRST>
__global__ void __launch_bounds__(256) ana_kernel(AnaArgs A) {
  extern __shared__ float smem[];
  const int id = blockIdx.x;
  int b = 0;
  while (b < kBases && id >= A.wg_prefix[b + 1]) ++b;
  const int wg = id - A.wg_prefix[b];
  switch (b) {
    case 0: ana_basis<2, E>(A, A.b[0], wg, smem); break;
    case 1: ana_basis<4, E>(A, A.b[1], wg, smem); break;
    case 2: ana_basis<6, E>(A, A.b[2], wg, smem); break;
    case 3: ana_basis<8, E>(A, A.b[3], wg, smem); break;
    case 4: ana_basis<10, E>(A, A.b[4], wg, smem); break;
    case 5: ana_basis<12, E>(A, A.b[5], wg, smem); break;
    case 6: ana_basis<14, E>(A, A.b[6], wg, smem); break;
    case 7: ana_basis<16, E>(A, A.b[7], wg, smem); break;
    default: ana_dirac<E>(A, A.b[8], wg); break;
  }
}

int launch_analysis(const AnaArgs &a, int nthreads, int lds_floats, int E, bool first, void *stream) {
  const int nwg = a.wg_prefix[kBases + 1];
  if (nwg <= 0) return FHS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t lds = static_cast<size_t>(lds_floats) * sizeof(float);
  if (E == 2) {
    if (first)
      hipLaunchKernelGGL((ana_kernel<2, true>), dim3(nwg), dim3(nthreads), lds, s, a);
    else
      hipLaunchKernelGGL((ana_kernel<2, false>), dim3(nwg), dim3(nthreads), lds, s, a);
  } else {
    if (first)
      hipLaunchKernelGGL((ana_kernel<1, true>), dim3(nwg), dim3(nthreads), lds, s, a);
    else
      hipLaunchKernelGGL((ana_kernel<1, false>), dim3(nwg), dim3(nthreads), lds, s, a);
  }
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("analysis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

// ---------------------------------------------------------------- synthesis
//
// Adjoint of one level (exact transpose of the analysis above).  An output
// sample x = 2k + px receives sum_{i < L/2} f[2i + 1 - px] c[k + i], so a thread
// owning coefficient column k produces both output columns 2k and 2k+1 and both
// output rows 2k' and 2k'+1 from the coefficient rows k' .. k' + L/2 - 1 held in
// a register ring.

// Loads coefficient row k of the four bands (columns kx0 .. kx0+segc-1).
__device__ __forceinline__ void syn_load_row(const SynBand &B, int k, int kx0, int segn, int L, float *dst) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int64_t rowlen = static_cast<int64_t>(B.Kx) * L;
  const int64_t base = static_cast<int64_t>(k) * rowlen;
  const int64_t c0 = static_cast<int64_t>(kx0) * L;
  const bool kok = k >= 0 && k < B.Ky;
  const float *src[4] = {B.ll, B.lh, B.hl, B.hh};
#pragma unroll
  for (int band = 0; band < 4; ++band) {
    const float *sp = src[band] + base;
    float *dp = dst + band * segn;
    for (int i = tid; i < segn; i += nth) {
      const int64_t gi = c0 + i;
      dp[i] = (kok && gi < rowlen) ? sp[gi] : 0.0f;
    }
  }
}

// x-adjoint of the current row for both output parities.
template <int NTAP>
__device__ __forceinline__ void syn_xadj(const SynBand &B, const float *buf, int segn, int off, int L,
                                         float &lo0, float &lo1, float &hi0, float &hi1) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
  lo0 = lo1 = hi0 = hi1 = 0.0f;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float cll = buf[off + i * L];
    const float clh = buf[segn + off + i * L];
    const float chl = buf[2 * segn + off + i * L];
    const float chh = buf[3 * segn + off + i * L];
    // even output column (px = 0): taps 2i+1 ; odd (px = 1): taps 2i
    lo0 = fmaf(T::h[2 * i + 1], cll, fmaf(T::g[2 * i + 1], clh, lo0));
    lo1 = fmaf(T::h[2 * i], cll, fmaf(T::g[2 * i], clh, lo1));
    hi0 = fmaf(T::h[2 * i + 1], chl, fmaf(T::g[2 * i + 1], chh, hi0));
    hi1 = fmaf(T::h[2 * i], chl, fmaf(T::g[2 * i], chh, hi1));
  }
}

template <int NTAP>
__device__ __forceinline__ void syn_basis(const SynArgs &A, const SynBand &B, int wg, float *buf) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % Lcp, grp = tid / Lcp, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int strip = wg % B.strips, yb = wg / B.strips;
  const int kx0 = strip * A.tk;
  const int y0 = yb * A.ty;
  const int y1 = min(y0 + A.ty, B.ny);
  const int segn = (A.tk + H - 1) * L;
  const int ks = y0 / 2;
  const int nout = (y1 - 1) / 2 - ks + 1;
  const int nk = nout + H - 1;
  const int off = kq * L + p;
  const int x = 2 * (kx0 + kq);

  float rlo[2][H], rhi[2][H];
#pragma unroll
  for (int i = 0; i < H; ++i) rlo[0][i] = rlo[1][i] = rhi[0][i] = rhi[1][i] = 0.0f;

  for (int r0 = 0; r0 < nk; r0 += H) {
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int r = r0 + u;
      if (r < nk) {
        __syncthreads();
        syn_load_row(B, ks + r, kx0, segn, L, buf);
        __syncthreads();
        syn_xadj<NTAP>(B, buf, segn, off, L, rlo[0][u], rlo[1][u], rhi[0][u], rhi[1][u]);
        if (r >= H - 1) {
          const int kp = ks + r - (H - 1);
#pragma unroll
          for (int py = 0; py < 2; ++py) {
            const int y = 2 * kp + py;
#pragma unroll
            for (int px = 0; px < 2; ++px) {
              float v = 0.0f;
#pragma unroll
              for (int i = 0; i < H; ++i) {
                const int s = (u - (H - 1) + i + H) % H;
                const int m = 2 * i + 1 - py;
                v = fmaf(T::h[m], rlo[px][s], fmaf(T::g[m], rhi[px][s], v));
              }
              if (lv && y < y1 && x + px < B.nx)
                B.out[(static_cast<int64_t>(y) * B.nx + x + px) * L + p] = v;
            }
          }
        }
      }
    }
  }
}

__global__ void __launch_bounds__(256) syn_kernel(SynArgs A) {
  extern __shared__ float smem[];
  const int id = blockIdx.x;
  int b = 0;
  while (b < kBases - 1 && id >= A.wg_prefix[b + 1]) ++b;
  const int wg = id - A.wg_prefix[b];
  switch (b) {
    case 0: syn_basis<2>(A, A.b[0], wg, smem); break;
    case 1: syn_basis<4>(A, A.b[1], wg, smem); break;
    case 2: syn_basis<6>(A, A.b[2], wg, smem); break;
    case 3: syn_basis<8>(A, A.b[3], wg, smem); break;
    case 4: syn_basis<10>(A, A.b[4], wg, smem); break;
    case 5: syn_basis<12>(A, A.b[5], wg, smem); break;
    case 6: syn_basis<14>(A, A.b[6], wg, smem); break;
    default: syn_basis<16>(A, A.b[7], wg, smem); break;
  }
}

int launch_synthesis(const SynArgs &a, int nthreads, int lds_floats, void *stream) {
  const int nwg = a.wg_prefix[kBases];
  if (nwg <= 0) return FHS_OK;
  hipLaunchKernelGGL(syn_kernel, dim3(nwg), dim3(nthreads), static_cast<size_t>(lds_floats) * sizeof(float),
                     static_cast<hipStream_t>(stream), a);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("synthesis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

// ---------------------------------------------------------------- final level
//
// Level 1 of all eight bases plus the Dirac basis, summed into the image in
// a fixed order (deterministic, no atomics).  Each basis keeps its own ring; at
// output step s the basis needs coefficient row ks + s + L_b/2 - 1, so every
// basis starts L_b/2 - 1 steps before the first output.

// Bases [0, kFinalSplit) go in the first final-level pass, the rest in the second.
constexpr int kFinalSplit = FHS_FINAL_SPLIT;

template <int NTAP>
struct Ring {
  float lo[2][NTAP / 2], hi[2][NTAP / 2];
};

template <int NTAP>
__device__ __forceinline__ void fin_push(const SynBand &B, const float *buf, int segn, int off, int L, Ring<NTAP> &R) {
  constexpr int H = NTAP / 2;
#pragma unroll
  for (int i = 0; i + 1 < H; ++i) {
    R.lo[0][i] = R.lo[0][i + 1];
    R.lo[1][i] = R.lo[1][i + 1];
    R.hi[0][i] = R.hi[0][i + 1];
    R.hi[1][i] = R.hi[1][i + 1];
  }
  syn_xadj<NTAP>(B, buf, segn, off, L, R.lo[0][H - 1], R.lo[1][H - 1], R.hi[0][H - 1], R.hi[1][H - 1]);
}

template <int NTAP>
__device__ __forceinline__ void fin_out(const Ring<NTAP> &R, float acc[2][2]) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
#pragma unroll
  for (int py = 0; py < 2; ++py)
#pragma unroll
    for (int px = 0; px < 2; ++px) {
      float v = 0.0f;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int m = 2 * i + 1 - py;
        v = fmaf(T::h[m], R.lo[px][i], fmaf(T::g[m], R.hi[px][i], v));
      }
      acc[py][px] += v;
    }
}

template <int NTAP>
__device__ __forceinline__ void fin_zero(Ring<NTAP> &R) {
#pragma unroll
  for (int i = 0; i < NTAP / 2; ++i) R.lo[0][i] = R.lo[1][i] = R.hi[0][i] = R.hi[1][i] = 0.0f;
}

// The rings of bases b .. BEND-1 (basis b has 2(b+1) taps).
template <int b, int BEND>
struct RingSet {
  Ring<2 * (b + 1)> r;
  RingSet<b + 1, BEND> next;
  __device__ __forceinline__ void zero() {
    fin_zero(r);
    next.zero();
  }
  // row step s: basis b holds rows ks + s .. ks + s + b once s >= -b
  __device__ __forceinline__ void load(const SynFinalArgs &A, int s, int ks, int kx0, int L, float *lds) {
    if (s >= -b) syn_load_row(A.b[b], ks + s + b, kx0, (A.tk + b) * L, L, lds);
    next.load(A, s, ks, kx0, L, lds + 4 * (A.tk + b) * L);
  }
  __device__ __forceinline__ void push(const SynFinalArgs &A, int s, int off, int L, const float *lds) {
    if (s >= -b) fin_push<2 * (b + 1)>(A.b[b], lds, (A.tk + b) * L, off, L, r);
    __builtin_amdgcn_sched_barrier(0);
    next.push(A, s, off, L, lds + 4 * (A.tk + b) * L);
  }
  __device__ __forceinline__ void out(float acc[2][2]) {
    fin_out<2 * (b + 1)>(r, acc);
    next.out(acc);
  }
};

template <int BEND>
struct RingSet<BEND, BEND> {
  __device__ __forceinline__ void zero() {}
  __device__ __forceinline__ void load(const SynFinalArgs &, int, int, int, int, float *) {}
  __device__ __forceinline__ void push(const SynFinalArgs &, int, int, int, const float *) {}
  __device__ __forceinline__ void out(float[2][2]) {}
};

// Bases B0 .. B1-1 of level 1 summed into the image; FIRST also adds the Dirac
// basis and applies beta, later groups accumulate (fixed order: deterministic).
template <int B0, int B1, bool FIRST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FHS_FINAL_WPE))) syn_final_kernel(SynFinalArgs A) {
  extern __shared__ float smem[];
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  const int lane = tid % Lcp, grp = tid / Lcp, c = grp % C, kq = grp / C;
  const bool lv = lane < Lc;
  const int p = c * Lc + lane;
  const int ch = c + lane * C;
  const int strip = blockIdx.x % A.strips, yb = blockIdx.x / A.strips;
  const int kx0 = strip * A.tk;
  const int y0 = yb * A.ty;
  const int y1 = min(y0 + A.ty, A.ny);
  const int ks = y0 / 2;
  const int nout = (y1 - 1) / 2 - ks + 1;
  const int x = 2 * (kx0 + kq);
  const int off = kq * L + p;
  RingSet<B0, B1> R;
  R.zero();
  const float scale = A.alpha * (1.0f / 3.0f);

  for (int s = -(B1 - 1); s < nout; ++s) {
    __syncthreads();
    R.load(A, s, ks, kx0, L, smem);
    __syncthreads();
    R.push(A, s, off, L, smem);
    if (s >= 0) {
      float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
      R.out(acc);
      const int kp = ks + s;
#pragma unroll
      for (int py = 0; py < 2; ++py) {
        const int y = 2 * kp + py;
#pragma unroll
        for (int px = 0; px < 2; ++px) {
          if (lv && y < y1 && x + px < A.nx) {
            const int64_t pix = static_cast<int64_t>(y) * A.nx + x + px;
            float *dst = A.x + pix * L + ch;
            if (FIRST) {
              const float v = acc[py][px] + A.dirac[pix * L + p];
              *dst = A.beta != 0.0f ? fmaf(A.beta, *dst, scale * v) : scale * v;
            } else {
              *dst = fmaf(scale, acc[py][px], *dst);
            }
          }
        }
      }
    }
  }
}

size_t final_lds_bytes(const SynFinalArgs &a, int b0, int b1) {
  size_t n = 0;
  for (int b = b0; b < b1; ++b) n += static_cast<size_t>(4) * (a.tk + b) * a.L;
  return n * sizeof(float);
}

// group 0: bases [0, kFinalSplit) + Dirac (applies beta); group 1: the rest.
int launch_synthesis_final(const SynFinalArgs &a, int nthreads, int group, void *stream) {
  const int nwg = a.strips * a.yblocks;
  if (nwg <= 0) return FHS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (group == 0)
    hipLaunchKernelGGL((syn_final_kernel<0, kFinalSplit, true>), dim3(nwg), dim3(nthreads),
                       final_lds_bytes(a, 0, kFinalSplit), s, a);
  else
    hipLaunchKernelGGL((syn_final_kernel<kFinalSplit, kBases, false>), dim3(nwg), dim3(nthreads),
                       final_lds_bytes(a, kFinalSplit, kBases), s, a);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("final synthesis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

}  // namespace fhs
