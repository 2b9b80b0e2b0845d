// Weighted nuclear-norm dual update for gfx950 (Alg. 2, the
// nuclear-norm dual update and facet back-projection; SVT of Table 1).
//
// For facet f (sub-cube c, spatial facet q) with Z = P_f + D_q S~_q Xcheck_c
// (N~_q x L_c):
//   nuc_gram : G = Z^T Z, FP64 MFMA (v_mfma_f64_16x16x4) on Z formed in FP64
//              from the FP32 inputs; one partial Gram per (facet, row chunk).
//   nuc_eig  : one workgroup per facet sums its partials (fixed order) and
//              diagonalises G = V Lambda V^T by parallel cyclic Jacobi in LDS
//              (FP64); s_j = sqrt(max(lambda_j, 0)) in descending order, t_j =
//              (mu_bar_f / zeta) theta_bar_{f,j}, h_j = min(1, t_j / s_j) (1 if
//              s_j = 0), K = V Diag(h) V^T.
//   nuc_recon: P_f <- Z K = U Diag(min(s_j, t_j)) V^T (U is never formed), FP64
//              MFMA, written in place.
//   nuc_gather: grad = beta grad + zeta sum_f S~_q^T D_q P_f, each pixel summing
//              the (at most four) facets that cover it in a fixed order.
// The window D_q is evaluated on the fly: weight 1 on the tile, a rising ramp
// (k+1)/(o+1) on the facet's own top/left border and the complementary falling
// ramp on the last o pixels of its tile (Sec. 2.4.2).
#include <hip/hip_runtime.h>

#include "fhs_internal.h"

namespace fhs {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kRB = 64;  // facet rows staged in LDS per step

struct FacetView {
  int c, sy, sx, wy0, wx0, hy, hx;
  int64_t poff, rows;
};

__device__ __forceinline__ FacetView facet_view(const NucGeom &g, int f) {
  FacetView F;
  const int Q = g.qy * g.qx;
  F.c = f / Q;
  const int q = f - F.c * Q;
  F.sy = q / g.qx;
  F.sx = q - F.sy * g.qx;
  F.wy0 = F.sy > 0 ? g.ty[F.sy] - g.oy : g.ty[F.sy];
  F.wx0 = F.sx > 0 ? g.tx[F.sx] - g.ox : g.tx[F.sx];
  F.hy = g.ty[F.sy + 1] - F.wy0;
  F.hx = g.tx[F.sx + 1] - F.wx0;
  F.rows = static_cast<int64_t>(F.hy) * F.hx;
  F.poff = F.c * g.p_sub +
           static_cast<int64_t>(g.Lc) * (static_cast<int64_t>(g.py[F.sy]) * g.px[g.qx] +
                                         static_cast<int64_t>(F.hy) * g.px[F.sx]);
  return F;
}

// 1D apodisation weight of local index i in the window of facet s (length len).
__device__ __forceinline__ double ramp(int i, int s, int Q, int o, int len) {
  if (s > 0 && i < o) return static_cast<double>(i + 1) / static_cast<double>(o + 1);
  if (s < Q - 1 && i >= len - o) return 1.0 - static_cast<double>(i - (len - o) + 1) / static_cast<double>(o + 1);
  return 1.0;
}

// Stages rows [r0, r0 + kRB) of Z (FP64, zero padded to W columns) into LDS.
// The first kRB threads resolve each row's pixel and window weight once
// (rinfo_pix / rinfo_d, kRB entries each); every element then needs no
// division.  The caller synchronises before and after.
template <int W>
__device__ __forceinline__ void stage_z(const NucArgs &A, const FacetView &F, int64_t r0, int64_t r_end, double *zs,
                                       int64_t *rinfo_pix, double *rinfo_d) {
  const NucGeom &g = A.g;
  if (threadIdx.x < kRB) {
    const int64_t r = r0 + threadIdx.x;
    int64_t pix = -1;
    double d = 0.0;
    if (r < r_end) {
      const int ri = static_cast<int>(r);  // facet rows fit in 32 bits
      const int yy = ri / F.hx, xx = ri - yy * F.hx;
      d = ramp(yy, F.sy, g.qy, g.oy, F.hy) * ramp(xx, F.sx, g.qx, g.ox, F.hx);
      pix = static_cast<int64_t>(F.wy0 + yy) * g.nx + (F.wx0 + xx);
    }
    rinfo_pix[threadIdx.x] = pix;
    rinfo_d[threadIdx.x] = d;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kRB * W; idx += blockDim.x) {
    const int rr = idx / W, l = idx % W;
    const int64_t pix = rinfo_pix[rr];
    double z = 0.0;
    if (pix >= 0 && l < g.Lc) {
      const double xv = static_cast<double>(A.x[pix * g.L + F.c + l * g.C]);
      const double pv = A.p ? static_cast<double>(A.p[F.poff + (r0 + rr) * g.Lc + l]) : 0.0;
      z = pv + rinfo_d[rr] * xv;
    }
    zs[rr * (W + 1) + l] = z;
  }
}

template <int NB>
__global__ void __launch_bounds__(256) nuc_gram_kernel(NucArgs A) {
  constexpr int W = NB * 16;
  constexpr int NPAIR = NB * (NB + 1) / 2;
  constexpr int PPW = (NPAIR + 3) / 4;
  __shared__ double zs[kRB * (W + 1)];
  __shared__ int64_t rinfo_pix[kRB];
  __shared__ double rinfo_d[kRB];
  const int f = blockIdx.y, chunk = blockIdx.x;
  const FacetView F = facet_view(A.g, f);
  const int64_t r_begin = static_cast<int64_t>(chunk) * A.chunk_rows;
  if (r_begin >= F.rows) return;
  const int64_t r_end = min(r_begin + A.chunk_rows, F.rows);
  const int wave = threadIdx.x / 64, ln = threadIdx.x % 64;
  int bi[PPW], bj[PPW];
  bool act[PPW];
#pragma unroll
  for (int t = 0; t < PPW; ++t) {
    const int idx = wave + 4 * t;
    act[t] = idx < NPAIR;
    int k = 0;
    bi[t] = bj[t] = 0;
    for (int a = 0; a < NB; ++a)
      for (int b = a; b < NB; ++b) {
        if (k == idx) {
          bi[t] = a;
          bj[t] = b;
        }
        ++k;
      }
  }
  v4d acc[PPW];
#pragma unroll
  for (int t = 0; t < PPW; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int64_t rb = r_begin; rb < r_end; rb += kRB) {
    __syncthreads();
    stage_z<W>(A, F, rb, r_end, zs, rinfo_pix, rinfo_d);
    __syncthreads();
#pragma unroll 4
    for (int k4 = 0; k4 < kRB / 4; ++k4) {
      const double *row = zs + (k4 * 4 + ln / 16) * (W + 1) + (ln % 16);
#pragma unroll
      for (int t = 0; t < PPW; ++t)
        if (act[t]) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * bi[t]], row[16 * bj[t]], acc[t], 0, 0, 0);
    }
  }
  double *out = A.gram + (static_cast<int64_t>(f) * A.chunks + chunk) * A.lc16 * A.lc16;
#pragma unroll
  for (int t = 0; t < PPW; ++t)
    if (act[t])
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // v_mfma_f64_16x16x4f64 result layout: lane holds D[4 v + lane / 16][lane % 16]
        const int i = 16 * bi[t] + 4 * v + ln / 16, j = 16 * bj[t] + ln % 16;
        out[i * A.lc16 + j] = acc[t][v];
      }
}

__device__ __forceinline__ void rr_pair(int r, int k, int n2, int &p, int &q) {
  // circle method: player 0 fixed, players 1..n2-1 rotate
  const int m = n2 - 1;
  if (k == 0) {
    p = 0;
    q = 1 + r % m;
  } else {
    p = 1 + (r + k) % m;
    q = 1 + (r - k + m) % m;
  }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < static_cast<int>(blockDim.x / 64); ++w) s += red[w];
  return s;
}

__global__ void __launch_bounds__(256) nuc_eig_kernel(NucArgs A) {
  __shared__ double Am[kMaxLc][kMaxLc + 1];
  __shared__ double Vm[kMaxLc][kMaxLc + 1];
  __shared__ double cs_c[kMaxLc / 2], cs_s[kMaxLc / 2];
  __shared__ int cs_p[kMaxLc / 2], cs_q[kMaxLc / 2];
  __shared__ double lam[kMaxLc], hv[kMaxLc];
  __shared__ int rank[kMaxLc];
  __shared__ double red[4];
  const NucGeom &g = A.g;
  const int f = blockIdx.x;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int n = g.Lc, n2 = n + (n & 1);
  const FacetView F = facet_view(g, f);
  const int nch = static_cast<int>((F.rows + A.chunk_rows - 1) / A.chunk_rows);
  const double *gp = A.gram + static_cast<int64_t>(f) * A.chunks * A.lc16 * A.lc16;
  for (int idx = tid; idx < n2 * n2; idx += nth) {
    const int i = idx / n2, j = idx - (idx / n2) * n2;
    double s = 0.0;
    if (i < n && j < n) {
      const int ii = min(i, j), jj = max(i, j);
      for (int k = 0; k < nch; ++k) s += gp[static_cast<int64_t>(k) * A.lc16 * A.lc16 + ii * A.lc16 + jj];
    }
    Am[i][j] = s;
    Vm[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < n2 * n2; idx += nth) {
      const int i = idx / n2, j = idx - (idx / n2) * n2;
      const double a2 = Am[i][j] * Am[i][j];
      tot += a2;
      if (i != j) off += a2;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (!(off > 1e-30 * tot)) break;
    for (int r = 0; r < n2 - 1; ++r) {
      if (tid < n2 / 2) {
        int p, q;
        rr_pair(r, tid, n2, p, q);
        const double apq = Am[p][q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300) {
          const double th = (Am[q][q] - Am[p][p]) / (2.0 * apq);
          double t;
          if (fabs(th) > 1e150)
            t = 0.5 / th;
          else
            t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        cs_c[tid] = c;
        cs_s[tid] = s;
        cs_p[tid] = p;
        cs_q[tid] = q;
      }
      __syncthreads();
      for (int idx = tid; idx < (n2 / 2) * n2; idx += nth) {
        const int k = idx / n2, j = idx - (idx / n2) * n2;
        const int p = cs_p[k], q = cs_q[k];
        const double c = cs_c[k], s = cs_s[k];
        const double a = Am[p][j], b = Am[q][j];
        Am[p][j] = c * a - s * b;
        Am[q][j] = s * a + c * b;
      }
      __syncthreads();
      for (int idx = tid; idx < (n2 / 2) * n2; idx += nth) {
        const int k = idx / n2, i = idx - (idx / n2) * n2;
        const int p = cs_p[k], q = cs_q[k];
        const double c = cs_c[k], s = cs_s[k];
        const double a = Am[i][p], b = Am[i][q];
        Am[i][p] = c * a - s * b;
        Am[i][q] = s * a + c * b;
        const double va = Vm[i][p], vb = Vm[i][q];
        Vm[i][p] = c * va - s * vb;
        Vm[i][q] = s * va + c * vb;
      }
      __syncthreads();
    }
  }
  if (tid < n) lam[tid] = Am[tid][tid];
  __syncthreads();
  if (tid < n) {
    int rk = 0;
    for (int j = 0; j < n; ++j)
      if (lam[j] > lam[tid] || (lam[j] == lam[tid] && j < tid)) ++rk;
    rank[tid] = rk;
    const double sig = sqrt(fmax(lam[tid], 0.0));
    A.sig[static_cast<int64_t>(f) * n + rk] = sig;
    if (A.mode == 0) {
      const double t = A.mu_bar[f] * A.inv_zeta * A.theta_bar[static_cast<int64_t>(f) * n + rk];
      hv[tid] = sig > 0.0 ? fmin(1.0, t / sig) : 1.0;
    } else {
      const double ub = A.mu_bar[f];
      A.theta_bar_out[static_cast<int64_t>(f) * n + rk] = ub / (sig + ub);
    }
  }
  __syncthreads();
  if (A.mode == 0) {
    double *K = A.kmat + static_cast<int64_t>(f) * A.lc16 * A.lc16;
    for (int idx = tid; idx < A.lc16 * A.lc16; idx += nth) {
      const int i = idx / A.lc16, j = idx - (idx / A.lc16) * A.lc16;
      double s = 0.0;
      if (i < n && j < n)
        for (int k = 0; k < n; ++k) s += Vm[i][k] * hv[k] * Vm[j][k];
      K[idx] = s;
    }
  }
}

template <int NB>
__global__ void __launch_bounds__(256) nuc_recon_kernel(NucArgs A) {
  constexpr int W = NB * 16;
  __shared__ double Ks[W * (W + 1)];
  __shared__ double zs[kRB * (W + 1)];
  __shared__ int64_t rinfo_pix[kRB];
  __shared__ double rinfo_d[kRB];
  const int f = blockIdx.y;
  const FacetView F = facet_view(A.g, f);
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRB;
  if (r0 >= F.rows) return;
  const double *K = A.kmat + static_cast<int64_t>(f) * A.lc16 * A.lc16;
  for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
    const int i = idx / W, j = idx - (idx / W) * W;
    Ks[i * (W + 1) + j] = K[i * A.lc16 + j];
  }
  stage_z<W>(A, F, r0, F.rows, zs, rinfo_pix, rinfo_d);
  __syncthreads();
  const int wave = threadIdx.x / 64, ln = threadIdx.x % 64;
  const int nb = wave;  // 16-row block of the 64 staged rows
  const int64_t r = r0 + 16 * nb + ln % 16;
#pragma unroll
  for (int mb = 0; mb < NB; ++mb) {
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < W / 4; ++kk) {
      const int k = 4 * kk + ln / 16;
      // A[m][k] = K[k][m], B[k][n] = Z[n][k]  ->  D[m][n] = (Z K)[n][m]
      const double a = Ks[k * (W + 1) + 16 * mb + ln % 16];
      const double b = zs[(16 * nb + ln % 16) * (W + 1) + k];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (r < F.rows) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * mb + 4 * v + ln / 16;
        if (j < A.g.Lc) A.p[F.poff + r * A.g.Lc + j] = static_cast<float>(acc[v]);
      }
    }
  }
}

// Thread = one pixel and up to 4 channels; all loads of the thread (up to 4
// facets x 4 channels of P, and the previous gradient) are independent.
__global__ void __launch_bounds__(256) nuc_gather_kernel(GatherArgs A) {
  const NucGeom &g = A.g;
  const int ngrp = (g.L + 3) / 4;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t npix = static_cast<int64_t>(g.ny) * g.nx;
  const int64_t pix = t / ngrp;
  if (pix >= npix) return;
  const int ch0 = 4 * static_cast<int>(t - pix * ngrp);
  const int y = static_cast<int>(pix / g.nx), x = static_cast<int>(pix - static_cast<int64_t>(y) * g.nx);
  const int sy0 = static_cast<int>((static_cast<int64_t>(y + 1) * g.qy + g.ny - 1) / g.ny) - 1;
  const int sx0 = static_cast<int>((static_cast<int64_t>(x + 1) * g.qx + g.nx - 1) / g.nx) - 1;
  const int ncy = (sy0 + 1 < g.qy && y >= g.ty[sy0 + 1] - g.oy) ? 2 : 1;
  const int ncx = (sx0 + 1 < g.qx && x >= g.tx[sx0 + 1] - g.ox) ? 2 : 1;
  // the (at most four) covering facets of sub-cube 0: weight and P row offset
  double dk[4];
  int64_t rk[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int dy = k >> 1, dx = k & 1;
    dk[k] = 0.0;
    rk[k] = 0;
    if (dy < ncy && dx < ncx) {
      const FacetView F = facet_view(g, (sy0 + dy) * g.qx + (sx0 + dx));
      const int yy = y - F.wy0, xx = x - F.wx0;
      dk[k] = ramp(yy, F.sy, g.qy, g.oy, F.hy) * ramp(xx, F.sx, g.qx, g.ox, F.hx);
      rk[k] = F.poff + (static_cast<int64_t>(yy) * F.hx + xx) * g.Lc;
    }
  }
  float pv[4][4], gv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ch = ch0 + e;
    const bool ok = ch < g.L;
    const int c = ch % g.C, l = ch / g.C;
#pragma unroll
    for (int k = 0; k < 4; ++k) pv[e][k] = (ok && dk[k] != 0.0) ? A.p[c * g.p_sub + rk[k] + l] : 0.0f;
    gv[e] = (ok && A.beta != 0.0f) ? A.grad[pix * g.L + ch] : 0.0f;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ch = ch0 + e;
    if (ch < g.L) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) sum += dk[k] * static_cast<double>(pv[e][k]);
      const float v = static_cast<float>(A.zeta * sum);
      A.grad[pix * g.L + ch] = A.beta != 0.0f ? fmaf(A.beta, gv[e], v) : v;
    }
  }
}

static int check_launch(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string(what) + ": " + hipGetErrorString(err));
  return FHS_OK;
}

int launch_nuc_gram(const NucArgs &a, int nfacets, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(a.chunks, nfacets);
  switch (a.lc16 / 16) {
    case 1: hipLaunchKernelGGL(nuc_gram_kernel<1>, grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(nuc_gram_kernel<2>, grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(nuc_gram_kernel<3>, grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(nuc_gram_kernel<4>, grid, dim3(256), 0, s, a); break;
    default: return fail(FHS_EUNSUPPORTED, "more than 64 channels per sub-cube");
  }
  return check_launch("nuc_gram");
}

int launch_nuc_eig(const NucArgs &a, int nfacets, void *stream) {
  hipLaunchKernelGGL(nuc_eig_kernel, dim3(nfacets), dim3(256), 0, static_cast<hipStream_t>(stream), a);
  return check_launch("nuc_eig");
}

int launch_nuc_recon(const NucArgs &a, int nfacets, int rowblocks, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(rowblocks, nfacets);
  switch (a.lc16 / 16) {
    case 1: hipLaunchKernelGGL(nuc_recon_kernel<1>, grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(nuc_recon_kernel<2>, grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(nuc_recon_kernel<3>, grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(nuc_recon_kernel<4>, grid, dim3(256), 0, s, a); break;
    default: return fail(FHS_EUNSUPPORTED, "more than 64 channels per sub-cube");
  }
  return check_launch("nuc_recon");
}

int launch_nuc_gather(const GatherArgs &a, void *stream) {
  const int64_t total = static_cast<int64_t>(a.g.ny) * a.g.nx * ((a.g.L + 3) / 4);
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(nuc_gather_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), a);
  return check_launch("nuc_gather");
}

}  // namespace fhs
