// The measurement operator Phi = G F Z of one channel per image plane (Sec.
// 2.1, eq. model) and the data-fidelity dual update of Alg. 2 (Sec. 3.2:
// projection onto the l2 ball in the metric of a diagonal preconditioner by
// forward-backward sub-iterations), for gfx950.
//
// Grid conventions: K = 2 N points per axis; the image is centred on the
// grid origin (pixel n at index (n - N/2) mod K, times the scaling of Z);
// F is the unnormalised DFT with exp(-2 pi i k g / K), its adjoint the
// unnormalised inverse.  The forward path keeps the spectrum transposed
// ([channel][k2][k1]) after its second FFT pass, and the de-gridding reads it
// there; the adjoint path grids into that layout and transposes back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <string>

#include "data_internal.h"
#include "fhs_internal.h"

namespace fhs {
namespace data {

namespace {

__device__ __forceinline__ float2v cmul(float2v a, float2v b) {
  return float2v{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---------------------------------------------------------------- Z and Z^T
__global__ void __launch_bounds__(256) pad_kernel(PadArgs a) {
  const int64_t n = static_cast<int64_t>(a.L) * a.K1 * a.K2;
  // (K1 and K2 are powers of two: indices by shifts and masks)
  const int lk1 = __ffs(a.K1) - 1, lk2 = __ffs(a.K2) - 1;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int k2 = static_cast<int>(i & (a.K2 - 1));
    const int64_t r = i >> lk2;
    const int k1 = static_cast<int>(r & (a.K1 - 1));
    const int l = static_cast<int>(r >> lk1);
    const int n1 = (k1 < a.K1 / 2 ? k1 : k1 - a.K1) + a.ny / 2;
    const int n2 = (k2 < a.K2 / 2 ? k2 : k2 - a.K2) + a.nx / 2;
    float v = 0.0f;
    if (n1 >= 0 && n1 < a.ny && n2 >= 0 && n2 < a.nx)
      v = a.x[(static_cast<int64_t>(n1) * a.nx + n2) * a.L + l] * (a.s1[n1] * a.s2[n2]);
    a.grid[i] = float2v{v, 0.0f};
  }
}

__global__ void __launch_bounds__(256) crop_kernel(CropArgs a) {
  const int64_t n = static_cast<int64_t>(a.ny) * a.nx * a.L;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int l = static_cast<int>(i % a.L);
    const int64_t pix = i / a.L;
    const int n2 = static_cast<int>(pix % a.nx), n1 = static_cast<int>(pix / a.nx);
    int k1 = n1 - a.ny / 2, k2 = n2 - a.nx / 2;
    if (k1 < 0) k1 += a.K1;
    if (k2 < 0) k2 += a.K2;
    const float g = a.grid[(static_cast<int64_t>(l) * a.K1 + k1) * a.K2 + k2].x * (a.s1[n1] * a.s2[n2]);
    const float sc = a.scale ? static_cast<float>(a.scale[l]) : 1.0f;
    a.x[i] = a.beta != 0.0f ? fmaf(a.beta, a.x[i], sc * g) : sc * g;
  }
}

// ---------------------------------------------------------------- F, by rows
// Workgroups walk rows of K points (a power of two), each row copied into
// LDS and transformed by Stockham passes (self-sorting, so no bit reversal):
// floor(log4 K) radix-4 passes, then one radix-2 pass when log2 K is odd.
// A radix-4 pass over blocks of n = 4m points with stride s (s = 1, 4, 16, ...)
// maps butterfly b = p s + q (p < m, q < s), a_k = x[q + s (p + k m)], to
//   t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = (a1 - a3) i^(sign)
//   y[q + s 4p] = t0 + t2,  y[q + s (4p + 2)] = (t0 - t2) W^(2 p s),
//   y[q + s (4p + 1)] = (t1 + t3) W^(p s),  y[q + s (4p + 3)] = (t1 - t3) W^(3 p s)
// and the radix-2 pass (m = 1) maps b = p s + q to
//   y[q + s 2p] = x[q + s p] + x[q + s (p + 1)],  y[q + s (2p + 1)] = (x[q + s p] - x[q + s (p + 1)]) W^(p s),
// with W = exp(sign 2 pi i / K) from the table of exp(-2 pi i k / K), k < K/2
// (W^(k + K/2) = -W^k; conjugated for sign > 0).
__device__ __forceinline__ float2v twiddle(const float2v *tw, int k, int half, int sign) {
  float2v w = k < half ? tw[k] : float2v{-tw[k - half].x, -tw[k - half].y};
  if (sign > 0) w.y = -w.y;
  return w;
}

// A workgroup takes rows blockIdx.x, blockIdx.x + gridDim.x, ...: the next
// row's points are loaded into registers while the passes of the current one
// run, so the row loads overlap the transform.
constexpr int kFftMaxPer = kMaxGrid / 1024;  // points per thread and row, upper bound

__global__ void __launch_bounds__(1024) fft_rows_kernel(float2v *data, int64_t rows, int K, const float2v *tw,
                                                        int sign) {
  extern __shared__ float2v buf[];
  const int nthr = static_cast<int>(blockDim.x);
  // the twiddle table in LDS after the two row buffers, loaded once per workgroup
  float2v *twl = buf + 2 * K;
  for (int i = threadIdx.x; i < (K >> 1); i += nthr) twl[i] = tw[i];
  float2v pre[kFftMaxPer];
  auto fetch = [&](int64_t r) __attribute__((always_inline)) {
    const float2v *src = data + r * K;
#pragma unroll
    for (int t = 0; t < kFftMaxPer; ++t) {
      const int i = static_cast<int>(threadIdx.x) + t * nthr;
      if (i < K) pre[t] = src[i];
    }
  };
  int64_t r = blockIdx.x;
  if (r < rows) fetch(r);
  for (; r < rows; r += gridDim.x) {
    float2v *x = buf, *y = buf + K;
    __syncthreads();  // (the previous row has left the LDS)
#pragma unroll
    for (int t = 0; t < kFftMaxPer; ++t) {
      const int i = static_cast<int>(threadIdx.x) + t * nthr;
      if (i < K) x[i] = pre[t];
    }
    __syncthreads();
    if (r + gridDim.x < rows) fetch(r + gridDim.x);
    const int half = K >> 1;
    int ls = 0, n = K;  // log2 of the stride, points per block
    for (; n >= 4; n >>= 2, ls += 2) {
      const int m = n >> 2, s = 1 << ls;
      for (int b = threadIdx.x; b < (K >> 2); b += blockDim.x) {
        const int p = b >> ls, q = b & (s - 1);
        const float2v a0 = x[q + s * p], a1 = x[q + s * (p + m)], a2 = x[q + s * (p + 2 * m)],
                      a3 = x[q + s * (p + 3 * m)];
        const float2v t0{a0.x + a2.x, a0.y + a2.y}, t1{a0.x - a2.x, a0.y - a2.y};
        const float2v t2{a1.x + a3.x, a1.y + a3.y}, d{a1.x - a3.x, a1.y - a3.y};
        // d i^(sign): times -i (forward) or +i (inverse)
        const float2v t3 = sign > 0 ? float2v{-d.y, d.x} : float2v{d.y, -d.x};
        const int e = p << ls;  // exponent p s
        y[q + s * 4 * p] = float2v{t0.x + t2.x, t0.y + t2.y};
        y[q + s * (4 * p + 1)] = cmul(float2v{t1.x + t3.x, t1.y + t3.y}, twiddle(twl, e, half, sign));
        y[q + s * (4 * p + 2)] = cmul(float2v{t0.x - t2.x, t0.y - t2.y}, twiddle(twl, 2 * e, half, sign));
        y[q + s * (4 * p + 3)] = cmul(float2v{t1.x - t3.x, t1.y - t3.y}, twiddle(twl, 3 * e, half, sign));
      }
      __syncthreads();
      float2v *t = x;
      x = y;
      y = t;
    }
    if (n == 2) {
      const int s = 1 << ls;
      for (int b = threadIdx.x; b < half; b += blockDim.x) {
        const int p = b >> ls, q = b & (s - 1);
        const float2v u = x[q + s * p], v = x[q + s * (p + 1)];
        y[q + s * 2 * p] = float2v{u.x + v.x, u.y + v.y};
        y[q + s * (2 * p + 1)] = cmul(float2v{u.x - v.x, u.y - v.y}, twiddle(twl, p << ls, half, sign));
      }
      __syncthreads();
      x = y;
    }
    float2v *row = data + r * K;
    for (int i = threadIdx.x; i < K; i += blockDim.x) row[i] = x[i];
  }
}

// out plane [Cc][R] = transpose of in plane [R][Cc], through 32 x 32 LDS tiles
__global__ void __launch_bounds__(256) transpose_kernel(const float2v *in, float2v *out, int R, int Cc) {
  __shared__ float2v tile[32][33];
  const int64_t plane = static_cast<int64_t>(blockIdx.z) * R * Cc;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + j, c = c0 + tx;
    if (r < R && c < Cc) tile[j][tx] = in[plane + static_cast<int64_t>(r) * Cc + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int c = c0 + j, r = r0 + tx;
    if (r < R && c < Cc) out[plane + static_cast<int64_t>(c) * R + r] = tile[tx][j];
  }
}

__global__ void __launch_bounds__(256) fill_zero_kernel(float2v *d, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    d[i] = float2v{0.0f, 0.0f};
}

// ---------------------------------------------------------------- G and G^H
// One thread per visibility: the J x J grid points from its first indices,
// wrapped modulo K, weights psi(t1 - k1) psi(t2 - k2) (FP64 accumulation).
// Threads take the visibilities in the gridding order (sorted by channel and
// grid tile), so that neighbouring threads read neighbouring grid points
// through the caches; each result goes to its visibility's own slot.
__global__ void __launch_bounds__(256) degrid_kernel(InterpArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.m) return;
  const int64_t j = a.perm[i];
  const VisInfo vi = a.info[j];
  const float *w = a.w + j * 2 * kKbWidth;
  const float2v *plane = a.spec + static_cast<int64_t>(vi.chan) * a.K1 * a.K2;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < kKbWidth; ++b) {
    int k2 = vi.k2 + b;
    if (k2 >= a.K2) k2 -= a.K2;
    const float2v *rowp = plane + static_cast<int64_t>(k2) * a.K1;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int c = 0; c < kKbWidth; ++c) {
      int k1 = vi.k1 + c;
      if (k1 >= a.K1) k1 -= a.K1;
      const float2v g = rowp[k1];
      sr += static_cast<double>(w[c]) * g.x;
      si += static_cast<double>(w[c]) * g.y;
    }
    re += static_cast<double>(w[kKbWidth + b]) * sr;
    im += static_cast<double>(w[kKbWidth + b]) * si;
  }
  a.vis_out[j] = float2v{static_cast<float>(re), static_cast<float>(im)};
}

// Gridding (G^H) by work items: the visibilities of one channel whose first
// grid indices lie in one tile of kGridTile x kGridTile points (sorted on the
// host) accumulate into the tile and its 6-point halo in LDS, which is then
// added to the grid (one global atomic per touched point and item instead of
// 49 per visibility: the coverage concentrates many visibilities on few grid
// points).
//
// LDS atomic adds of floats run at a small fraction of the rate of integer
// ones here (measured about 0.2 against 3 to 5 T lane-adds per second), so the
// tile accumulates in 64-bit fixed point: each contribution w1 w2 v, formed in
// FP64, is scaled by 2^s and rounded to an integer below 2^51 in magnitude,
// s = 51 - e_v - wexp (the item's largest |v| component is below 2^e_v and
// every weight product below 2^wexp); a tile point then sums at most
// kGridChunk of them, below 2^62.  The rounding, at most 2^-52 of the largest
// possible contribution, is the only error; the integer sums are exact and do
// not depend on the order.  An item with a non-finite visibility adds in FP32
// instead, so that NaN and Inf reach the grid as they are.
constexpr int kTileExt = kGridTile + kKbWidth - 1;
constexpr double kRoundMagic = 6755399441055744.0;  // 1.5 * 2^52

// x rounded to the nearest integer, for |x| < 2^51: the low bits of x + 1.5 * 2^52
__device__ __forceinline__ long long round_fixed(double x) {
  return __double_as_longlong(x + kRoundMagic) - __double_as_longlong(kRoundMagic);
}

__global__ void __launch_bounds__(256) grid_kernel(InterpArgs a) {
  constexpr int T = kTileExt * kTileExt;
  __shared__ unsigned long long acc[2 * T];  // fixed point: re [0, T), im [T, 2T)
  __shared__ float wmax[256 / 64];
  __shared__ int wbad[256 / 64];
  float *tf = reinterpret_cast<float *>(acc);  // the FP32 form: re [0, T), im [T, 2T)
  const GridItem it = a.items[blockIdx.x];
  for (int e = threadIdx.x; e < 2 * T; e += blockDim.x) acc[e] = 0ull;
  // largest |v| component of the item, and whether all are finite
  float m = 0.0f;
  int bad = 0;
  for (int i = it.start + threadIdx.x; i < it.start + it.count; i += blockDim.x) {
    const float2v v = a.vis_in[a.perm[i]];
    const float ax = fabsf(v.x), ay = fabsf(v.y);
    bad |= !(ax <= 3.4e38f) || !(ay <= 3.4e38f);  // NaN or Inf (fmaxf would drop a NaN)
    m = fmaxf(m, fmaxf(ax, ay));
  }
  for (int o = 32; o > 0; o >>= 1) {
    m = fmaxf(m, __shfl_xor(m, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wmax[threadIdx.x >> 6] = m;
    wbad[threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  m = 0.0f;
  bad = 0;
  for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
    m = fmaxf(m, wmax[w]);
    bad |= wbad[w];
  }
  int ev = 0;
  frexpf(m, &ev);  // m < 2^ev
  const int sh = 51 - ev - a.wexp;
  const double scale = ldexp(1.0, sh);
  if (bad || m > 0.0f) {
    for (int i = it.start + threadIdx.x; i < it.start + it.count; i += blockDim.x) {
      const int64_t j = a.perm[i];
      const VisInfo vi = a.info[j];
      const float *w = a.w + j * 2 * kKbWidth;
      const float2v v = a.vis_in[j];
      const int r0 = vi.k1 - it.t1 * kGridTile, c0 = vi.k2 - it.t2 * kGridTile;  // in [0, kGridTile)
      float wr[2 * kKbWidth];
#pragma unroll
      for (int t = 0; t < 2 * kKbWidth; ++t) wr[t] = w[t];
      const double vx = static_cast<double>(v.x) * scale, vy = static_cast<double>(v.y) * scale;
      for (int b = 0; b < kKbWidth; ++b) {
        const float wb = wr[kKbWidth + b];
#pragma unroll
        for (int c = 0; c < kKbWidth; ++c) {
          const int e = (c0 + b) * kTileExt + r0 + c;
          if (bad) {
            const float ww = wb * wr[c];
            atomicAdd(&tf[e], ww * v.x);
            atomicAdd(&tf[T + e], ww * v.y);
          } else {
            const double ww = static_cast<double>(wb) * static_cast<double>(wr[c]);
            atomicAdd(&acc[e], static_cast<unsigned long long>(round_fixed(ww * vx)));
            atomicAdd(&acc[T + e], static_cast<unsigned long long>(round_fixed(ww * vy)));
          }
        }
      }
    }
  }
  __syncthreads();
  float2v *plane = a.grid + static_cast<int64_t>(it.chan) * a.K1 * a.K2;
  for (int e = threadIdx.x; e < T; e += blockDim.x) {
    float re, im;
    if (bad) {
      re = tf[e];
      im = tf[T + e];
    } else {
      re = static_cast<float>(ldexp(static_cast<double>(static_cast<long long>(acc[e])), -sh));
      im = static_cast<float>(ldexp(static_cast<double>(static_cast<long long>(acc[T + e])), -sh));
    }
    if (re == 0.0f && im == 0.0f) continue;
    const int cb = e / kTileExt, ra = e - cb * kTileExt;
    const int g2 = (it.t2 * kGridTile + cb) % a.K2, g1 = (it.t1 * kGridTile + ra) % a.K1;
    atomicAdd(&plane[static_cast<int64_t>(g2) * a.K1 + g1].x, re);
    atomicAdd(&plane[static_cast<int64_t>(g2) * a.K1 + g1].y, im);
  }
}

// ---------------------------------------------------------------- data dual
// The update of one channel (one data block) in passes over its visibilities,
// kDualBlocks workgroups per channel, each writing its partial sums (FP64, a
// fixed-order tree in LDS), then one workgroup per channel summing them in
// order:
//   pass 0: d2 = ||z - y||^2, r2 = ||y - Phi x||^2, max U   (z = v / U + Phi xcheck)
//           -> f = min(1, eps / sqrt(d2)) (p = P_B(z) = y + f (z - y)), gamma = 1 / max U
//   pass s = 1 .. n_sub: p = y + f (prev - y) (prev = z, then the stored q);
//           q = p - gamma U (p - z), stored; ||q - y||^2 -> f
//   last pass: p = y + f (prev - y); v <- U (z - p)
__device__ double block_sum(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float2v zval(const DualArgs &a, int64_t j) {
  const float2v v = a.v[j], c = a.yc[j];
  const float u = a.U[j];
  return float2v{v.x / u + c.x, v.y / u + c.y};
}

// mode 0: first pass; 1: a sub-iteration (first = 1 when prev is z); 2: the last pass
__global__ void __launch_bounds__(kDualThreads) dual_pass_kernel(DualArgs a, int mode, int first) {
  __shared__ double red[kDualThreads];
  const int l = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
  const int64_t c0 = a.voff[l], n = a.voff[l + 1] - c0;
  const int64_t len = (n + kDualBlocks - 1) / kDualBlocks;
  const int64_t j0 = c0 + blk * len, j1 = c0 + min(n, (blk + 1) * len);
  const double f = a.chs[4 * l], gamma = a.chs[4 * l + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t j = j0 + t; j < j1; j += blockDim.x) {
    const float2v z = zval(a, j), y = a.y[j];
    if (mode == 0) {
      const float2v yx = a.yx[j];
      const double dx = static_cast<double>(z.x) - y.x, dy = static_cast<double>(z.y) - y.y;
      const double ex = static_cast<double>(y.x) - yx.x, ey = static_cast<double>(y.y) - yx.y;
      s0 += dx * dx + dy * dy;
      s1 += ex * ex + ey * ey;
      s2 = fmax(s2, static_cast<double>(a.U[j]));
      continue;
    }
    const float2v prev = first ? z : a.p[j];
    const float2v p{static_cast<float>(y.x + f * (static_cast<double>(prev.x) - y.x)),
                    static_cast<float>(y.y + f * (static_cast<double>(prev.y) - y.y))};
    const float u = a.U[j];
    if (mode == 1) {
      const float g = static_cast<float>(gamma) * u;
      const float2v q{p.x - g * (p.x - z.x), p.y - g * (p.y - z.y)};
      a.p[j] = q;
      const double dx = static_cast<double>(q.x) - y.x, dy = static_cast<double>(q.y) - y.y;
      s0 += dx * dx + dy * dy;
    } else {
      a.v[j] = float2v{u * (z.x - p.x), u * (z.y - p.y)};
    }
  }
  if (mode == 2) return;  // (uniform: no partial sums)
  s0 = block_sum(s0, red);
  if (mode == 0) {
    s1 = block_sum(s1, red);
    s2 = block_max(s2, red);
  }
  if (t == 0) {
    double *pp = a.part + (static_cast<int64_t>(l) * kDualBlocks + blk) * 4;
    pp[0] = s0;
    pp[1] = s1;
    pp[2] = s2;
  }
}

// one thread per channel: the workgroups' partial sums in order
__global__ void __launch_bounds__(64) dual_finalize_kernel(DualArgs a, int mode) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.L) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < kDualBlocks; ++b) {
    const double *pp = a.part + (static_cast<int64_t>(l) * kDualBlocks + b) * 4;
    s0 += pp[0];
    s1 += pp[1];
    s2 = fmax(s2, pp[2]);
  }
  const double eps = a.eps[l];
  a.chs[4 * l] = s0 > eps * eps ? eps / sqrt(s0) : 1.0;
  if (mode == 0) {
    a.chs[4 * l + 1] = s2 > 0.0 ? 1.0 / s2 : 0.0;
    a.chs[4 * l + 2] = sqrt(s1);
    if (a.residual) a.residual[l] = sqrt(s1);
  }
}

int check(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string(what) + ": " + hipGetErrorString(err));
  return FHS_OK;
}

unsigned grid_for(int64_t n, int threads) {
  const int64_t g = (n + threads - 1) / threads;
  return static_cast<unsigned>(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

int launch_pad(const PadArgs &a, void *stream) {
  const int64_t n = static_cast<int64_t>(a.L) * a.K1 * a.K2;
  hipLaunchKernelGGL(pad_kernel, dim3(grid_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), a);
  return check("nufft pad");
}

int launch_crop(const CropArgs &a, void *stream) {
  const int64_t n = static_cast<int64_t>(a.ny) * a.nx * a.L;
  hipLaunchKernelGGL(crop_kernel, dim3(grid_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), a);
  return check("nufft crop");
}

int launch_fft_rows(float2v *data, int64_t rows, int K, const float2v *tw, int sign, void *stream) {
  if (rows <= 0) return FHS_OK;
  if (K < 2 || K > kMaxGrid || (K & (K - 1)) != 0) return fail(FHS_EUNSUPPORTED, "FFT length must be a power of two");
  if (rows > 0x7fffffff) return fail(FHS_EUNSUPPORTED, "too many FFT rows");
  // (one radix-4 butterfly per thread and pass, up to 1024 threads; as many
  // workgroups as fit on the 256 CUs at once by LDS and by waves, each walking
  // its share of the rows)
  const int threads = K / 4 < 1024 ? (K / 4 < 64 ? 64 : K / 4) : 1024;
  const size_t lds = static_cast<size_t>(2 * K + K / 2) * sizeof(float2v);  // two row buffers, twiddles
  const int per_cu = std::max(1, std::min(static_cast<int>((160 * 1024) / lds), 32 / (threads / 64)));
  const int64_t nwg = std::min<int64_t>(rows, 256 * static_cast<int64_t>(per_cu));
  hipLaunchKernelGGL(fft_rows_kernel, dim3(static_cast<unsigned>(nwg)), dim3(threads), lds,
                     static_cast<hipStream_t>(stream), data, rows, K, tw, sign);
  return check("nufft fft rows");
}

int launch_transpose(const float2v *in, float2v *out, int R, int Cc, int planes, void *stream) {
  const dim3 grid((Cc + 31) / 32, (R + 31) / 32, planes);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), in, out, R, Cc);
  return check("nufft transpose");
}

int launch_fill_zero(float2v *data, int64_t n, void *stream) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), data,
                     n);
  return check("nufft fill");
}

int launch_degrid(const InterpArgs &a, void *stream) {
  if (a.m <= 0) return FHS_OK;
  hipLaunchKernelGGL(degrid_kernel, dim3(static_cast<unsigned>((a.m + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), a);
  return check("nufft degrid");
}

int launch_grid(const InterpArgs &a, void *stream) {
  if (a.n_items <= 0) return FHS_OK;
  if (a.n_items > 0x7fffffff) return fail(FHS_EUNSUPPORTED, "too many gridding work items");
  hipLaunchKernelGGL(grid_kernel, dim3(static_cast<unsigned>(a.n_items)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), a);
  return check("nufft grid");
}

int launch_data_dual(const DualArgs &a, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(kDualBlocks, a.L), fin((a.L + 63) / 64);
  hipLaunchKernelGGL(dual_pass_kernel, grid, dim3(kDualThreads), 0, s, a, 0, 1);
  hipLaunchKernelGGL(dual_finalize_kernel, fin, dim3(64), 0, s, a, 0);
  for (int it = 0; it < a.n_sub; ++it) {
    hipLaunchKernelGGL(dual_pass_kernel, grid, dim3(kDualThreads), 0, s, a, 1, it == 0 ? 1 : 0);
    hipLaunchKernelGGL(dual_finalize_kernel, fin, dim3(64), 0, s, a, 1);
  }
  hipLaunchKernelGGL(dual_pass_kernel, grid, dim3(kDualThreads), 0, s, a, 2, a.n_sub == 0 ? 1 : 0);
  return check("data dual update");
}

}  // namespace data
}  // namespace fhs
