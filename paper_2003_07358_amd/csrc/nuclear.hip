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

#include <type_traits>

#include "fhs_internal.h"
#include "lds_stage.h"

namespace fhs {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));  // four bfloat16 bit patterns

// float -> bfloat16 bits, rounding to nearest even (finite inputs)
__device__ __forceinline__ short bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return static_cast<short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}


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

// ---------------------------------------------------------------- staging
// A workgroup owns one spatial facet q and a chunk of its window rows, for
// every sub-cube at once (the cube is read once, whatever C).  It walks the
// chunk in segments of S consecutive pixels of one window row: the segment's
// X (S x L floats, one contiguous run of HBM) and, per sub-cube, its P rows
// (S x L_c floats, contiguous) are copied HBM -> LDS by buffer loads with LDS
// destination, one segment ahead into a double buffer; the window weight of
// each pixel is computed into LDS at the same time.
struct Seg {
  int y, s0, n;  // window row, first pixel of the segment, pixels in it
};

__device__ __forceinline__ Seg seg_of(int i, int y0, int nsx, int S, int hx) {
  Seg sg;
  sg.y = y0 + i / nsx;
  sg.s0 = (i - (i / nsx) * nsx) * S;
  sg.n = min(S, hx - sg.s0);
  return sg;
}

// words of one staging buffer: X [S][L] then P [C][S][L_c]
__device__ __forceinline__ int stage_words(const NucGeom &g, int S) { return S * (g.L + g.C * g.Lc); }

// Overlapping spectral facets (contiguous blocks): channel of column ch of
// block c (negative before the cube: a structural-zero column of the first
// block) and its spectral weight, the triangular ramp of the spatial window
// (Sec. 2.4.2) on the channel axis: rising over the so columns before the
// block (not for the first block), falling over the block's last so columns
// (not for the last block).
__device__ __forceinline__ int spec_chan(const NucGeom &g, int c, int ch) { return c * g.sb - g.so + ch; }
__device__ __forceinline__ double spec_weight(const NucGeom &g, int c, int ch) {
  if (c > 0 && ch < g.so) return static_cast<double>(ch + 1) / static_cast<double>(g.so + 1);
  if (c < g.C - 1 && ch >= g.Lc - g.so)
    return 1.0 - static_cast<double>(ch - (g.Lc - g.so) + 1) / static_cast<double>(g.so + 1);
  return 1.0;
}

__device__ __forceinline__ void issue_seg(const NucArgs &A, const FacetView &F, const Seg &sg, float *buf, double *dsh,
                                          bool with_p) {
  const NucGeom &g = A.g;
  const int S = A.seg, L = g.L, Lc = g.Lc;
  copy_span(A.x + (static_cast<int64_t>(F.wy0 + sg.y) * g.nx + F.wx0 + sg.s0) * L, sg.n * L, buf);
  if (with_p)
    for (int c = 0; c < g.C; ++c)
      copy_span(A.p + c * g.p_sub + F.poff + (static_cast<int64_t>(sg.y) * F.hx + sg.s0) * Lc, sg.n * Lc,
                buf + S * L + c * S * Lc);
  if (threadIdx.x < S) {
    const int i = threadIdx.x;
    dsh[i] = i < sg.n ? ramp(sg.y, F.sy, g.qy, g.oy, F.hy) * ramp(sg.s0 + i, F.sx, g.qx, g.ox, F.hx) : 0.0;
  }
}

// Z_c[r][ch] = P_c[r][ch] + D_r X[r][c + ch C] in FP64 (0 outside the segment
// and beyond L_c); SPEC: + D_r d_c(ch) X[r][c sb - so + ch] (overlapping
// spectral facets; P alone on structural-zero columns).
template <bool SPEC>
__device__ __forceinline__ double zval(const NucArgs &A, const float *buf, const double *dsh, int n, bool with_p,
                                       int c, int r, int ch) {
  const NucGeom &g = A.g;
  if (r >= n || ch >= g.Lc) return 0.0;
  const int S = A.seg, L = g.L;
  const double pv = with_p ? static_cast<double>(buf[S * L + (c * S + r) * g.Lc + ch]) : 0.0;
  if constexpr (SPEC) {
    const int chan = spec_chan(g, c, ch);
    return chan >= 0 ? fma(dsh[r] * spec_weight(g, c, ch), static_cast<double>(buf[r * L + chan]), pv) : pv;
  } else {
    const double xv = static_cast<double>(buf[r * L + c + ch * g.C]);
    return fma(dsh[r], xv, pv);
  }
}

constexpr int kMaxSeg = 64;  // pixels per segment (upper bound)

// One sub-cube with L a multiple of 4 (the common case): the X and P runs of a
// segment (n pixels x L floats, contiguous in HBM) are copied in 16-byte chunks
// into rows of Lp floats, X first, then P at word `preg`; chunk i covers the
// 4-float groups u = 64 i + lane, row u / (Lp / 4).  A row stride that is a
// multiple of 16 words would put the pixels an MFMA operand reads (same
// channel, rows 1 or 4 apart) in one LDS bank, so such strides get four words
// of padding.  The per-lane source offsets do not depend on the segment (rows
// past its end fall outside the run and read zero), so each wave computes
// those of its chunks i = wave + 4 t once.
__host__ __device__ __forceinline__ int one_stride(int L) { return L % 16 == 0 ? L + 4 : L; }
// floats of one staged array (X or P) of S pixels: whole 256-float copy chunks
__host__ __device__ __forceinline__ int one_region(int S, int L) { return (S * one_stride(L) + 255) / 256 * 256; }

// The Gram kernel stages through OneStage for one sub-cube without spectral
// overlap and L a multiple of 4.
__host__ __device__ __forceinline__ bool gram_one_stage(const NucGeom &g) {
  return g.C == 1 && !g.spec && g.L % 4 == 0;
}

struct OneStage {
  static constexpr int kMaxChunks = 5;  // 16-byte copy chunks per wave and array (ceil(17 / 4))
  int coff[kMaxChunks];
  int nchunk, preg, Lp;
  __device__ __forceinline__ void init(int S, int L, int wave, int ln) {
    Lp = one_stride(L);
    preg = one_region(S, L);
    const int gp = Lp / 4;
    nchunk = (S * gp + 63) / 64;
#pragma unroll
    for (int t = 0; t < kMaxChunks; ++t) {
      const int u = 64 * (wave + 4 * t) + ln, r = u / gp, gg = u - r * gp;
      coff[t] = (gg < L / 4 && r < S) ? (r * L + 4 * gg) * 4 : static_cast<int>(0x80000000u);
    }
  }
  // copies of segment sg (P too when with_p) and its window weights
  __device__ __forceinline__ void issue(const NucArgs &A, const FacetView &F, const Seg &sg, float *buf, double *dd,
                                        bool with_p, int wave) const {
    const NucGeom &g = A.g;
    const int L = g.L;
    const float *xs = A.x + (static_cast<int64_t>(F.wy0 + sg.y) * g.nx + F.wx0 + sg.s0) * L;
    const fhs_int32x4 rx = buffer_rsrc(xs, static_cast<unsigned>(sg.n * L * 4));
    fhs_int32x4 rp = rx;
    if (with_p) {
      const float *ps = A.p + F.poff + (static_cast<int64_t>(sg.y) * F.hx + sg.s0) * L;
      rp = buffer_rsrc(ps, static_cast<unsigned>(sg.n * L * 4));
    }
#pragma unroll
    for (int t = 0; t < kMaxChunks; ++t) {
      const int i = wave + 4 * t;
      if (i < nchunk) {
        fhs_raw_buffer_load_lds(rx, lds_words(buf + 256 * i), 16, coff[t], 0, 0, 0);
        if (with_p) fhs_raw_buffer_load_lds(rp, lds_words(buf + preg + 256 * i), 16, coff[t], 0, 0, 0);
      }
    }
    if (threadIdx.x < A.seg) {
      const int i = threadIdx.x;
      dd[i] = i < sg.n ? ramp(sg.y, F.sy, g.qy, g.oy, F.hy) * ramp(sg.s0 + i, F.sx, g.qx, g.ox, F.hx) : 0.0;
    }
  }
};

// block pairs (bi <= bj) of NB 16-channel blocks
template <int NB>
struct Pairs {
  static constexpr int n = NB * (NB + 1) / 2;
};

// Sub-cubes per Gram workgroup: about ten block pairs of accumulators.
template <int NB>
constexpr int gram_subcubes() {
  return Pairs<NB>::n >= 10 ? 1 : 10 / Pairs<NB>::n;
}

// Partial Grams of the chunk for sub-cubes [K blockIdx.z, K blockIdx.z + K).
// Wave w takes the groups of four rows k4 = w mod 4 of every segment; per row
// group and sub-cube the NB 16-channel columns of Z are formed once and feed
// the NB (NB + 1) / 2 block pairs.  The four waves' partials are summed in LDS
// in a fixed order at the end.
//
// BF16 (mixed-precision form): Z is formed in FP32, rounded to bfloat16 and
// multiplied on v_mfma_f32_16x16x16_bf16 with FP32 accumulation, in groups of
// 16 rows (lane l holds rows 4 (l / 16) .. + 3 of its channel l mod 16: the
// same operand serves as A = Z^T and B = Z, as in the FP64 form); the
// partials are summed across waves in FP64.
template <int NB, int K, bool BF16, bool SPEC = false>
__global__ void __launch_bounds__(256) nuc_gram_kernel(NucArgs A) {
  static_assert(!(BF16 && SPEC), "overlapping spectral facets run in the FP32 form only");
  using PR = Pairs<NB>;
  extern __shared__ float sm[];
  __shared__ double dsh[2][kMaxSeg];
  const NucGeom &g = A.g;
  const int q = A.q0 + blockIdx.y, chunk = blockIdx.x, Q = g.qy * g.qx;
  const FacetView F = facet_view(g, q);
  const int y0 = chunk * A.chunk_wrows;
  if (y0 >= F.hy) return;
  const int y1 = min(y0 + A.chunk_wrows, F.hy);
  const int S = A.seg, L = g.L;
  const int nsx = (F.hx + S - 1) / S, nseg = (y1 - y0) * nsx;
  const bool with_p = A.p != nullptr;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  const int c0 = blockIdx.z * K, nc = min(K, g.C - c0);
  // one sub-cube, L a multiple of 4: padded rows (OneStage), X row r at r Lp,
  // P row r at preg + r Lp; else X [S][L] then P [C][S][L_c]
  const bool one = gram_one_stage(g);
  OneStage st;
  st.init(S, L, wave, ln);
  const int BUF = one ? 2 * st.preg : stage_words(g, S);
  const int xrs = one ? st.Lp : L;  // X row stride
  auto issue = [&](const Seg &sg, float *buf, double *dd) __attribute__((always_inline)) {
    if (one)
      st.issue(A, F, sg, buf, dd, with_p, wave);
    else
      issue_seg(A, F, sg, buf, dd, with_p);
  };
  // word of P row r, channel ch of sub-cube c in a staging buffer
  auto pword = [&](int c, int r, int ch) __attribute__((always_inline)) {
    return one ? st.preg + r * st.Lp + ch : S * L + (c * S + r) * g.Lc + ch;
  };
  if (A.sel != nullptr) {  // randomized step: no selected facet among these sub-cubes
    bool any = false;
    for (int kc = 0; kc < nc; ++kc) any = any || A.sel[(c0 + kc) * Q + q] != 0;
    if (!any) return;
  }
  using Acc = typename std::conditional<BF16, v4f, v4d>::type;
  Acc acc[K][PR::n];
#pragma unroll
  for (int kc = 0; kc < K; ++kc)
#pragma unroll
    for (int t = 0; t < PR::n; ++t) acc[kc][t] = Acc{0, 0, 0, 0};

  issue(seg_of(0, y0, nsx, S, F.hx), sm, dsh[0]);
  for (int i = 0; i < nseg; ++i) {
    wait_loads_and_sync();
    if (i + 1 < nseg) issue(seg_of(i + 1, y0, nsx, S, F.hx), sm + ((i + 1) & 1) * BUF, dsh[(i + 1) & 1]);
    const float *buf = sm + (i & 1) * BUF;
    const double *d = dsh[i & 1];
    const int n = seg_of(i, y0, nsx, S, F.hx).n;
    if constexpr (BF16) {
      for (int k16 = wave; k16 < S / 16; k16 += 4) {
        const int rb = 16 * k16 + 4 * (ln / 16);
#pragma unroll
        for (int kc = 0; kc < K; ++kc) {
          if (kc < nc) {
            const int c = c0 + kc, ch0 = ln & 15;
            v4s z[NB];
            // unconditional reads (channel clamped into the sub-cube, rows
            // below S), then a select, as in the FP64 form
            float xv[NB][4], pv[NB][4];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const int ch = min(16 * b + ch0, g.Lc - 1);
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                xv[b][t] = buf[(rb + t) * xrs + c + ch * g.C];
                pv[b][t] = with_p ? buf[pword(c, rb + t, ch)] : 0.0f;
              }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const bool chv = 16 * b + ch0 < g.Lc;
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int r = rb + t;
                const bool ok = chv && r < n;
                const float zz = fmaf(static_cast<float>(d[r]), xv[b][t], pv[b][t]);
                z[b][t] = bf16_bits(ok ? zz : 0.0f);
              }
            }
            int t = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
              for (int bj = bi; bj < NB; ++bj, ++t)
                acc[kc][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(z[bi], z[bj], acc[kc][t], 0, 0, 0);
          }
        }
      }
    } else if (!SPEC && one) {
      // One sub-cube: the wave's row groups k4 = wave, wave + 4, ... taken two
      // per iteration, the reads of both issued first, so that the second
      // group's reads land while the first group's MFMAs run (the
      // accumulation order is that of the plain loop).  Any split of the rows
      // into groups of four gives the same Gram; with padded rows the four
      // rows k4 % 4 + 16 (k4 / 4) + 4 j, j = lane / 16, put the 64 words an
      // operand read takes in distinct LDS banks.
      const int ch0 = ln & 15;
      auto rows_of = [&](int k4) { return 16 * (k4 >> 2) + (k4 & 3) + 4 * (ln / 16); };
      auto load = [&](int r, float(&xv)[NB], float(&pv)[NB]) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          // (unconditional reads, channel clamped into the cube, rows below S)
          const int ch = min(16 * b + ch0, g.Lc - 1);
          xv[b] = buf[r * st.Lp + ch];
          pv[b] = with_p ? buf[st.preg + r * st.Lp + ch] : 0.0f;
        }
      };
      auto accumulate = [&](int r, const float(&xv)[NB], const float(&pv)[NB]) __attribute__((always_inline)) {
        const bool rv = r < n;
        const double dr = d[r];
        double z[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double zz = fma(dr, static_cast<double>(xv[b]), static_cast<double>(pv[b]));
          z[b] = (rv && 16 * b + ch0 < g.Lc) ? zz : 0.0;
        }
        int t = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NB; ++bj, ++t)
            acc[0][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[bi], z[bj], acc[0][t], 0, 0, 0);
      };
      for (int k4 = wave; k4 < S / 4; k4 += 8) {
        const bool two = k4 + 4 < S / 4;
        const int ra = rows_of(k4), rb = rows_of(k4 + 4);
        float xa[NB], pa[NB], xb[NB], pb[NB];
        load(ra, xa, pa);
        if (two) load(rb, xb, pb);
        accumulate(ra, xa, pa);
        if (two) accumulate(rb, xb, pb);
      }
    } else {
      for (int k4 = wave; k4 < S / 4; k4 += 4) {
        const int r = 4 * k4 + ln / 16;
        const bool rv = r < n;
        const double dr = d[r];
#pragma unroll
        for (int kc = 0; kc < K; ++kc) {
          if (kc < nc) {
            // Z[r][ch] = P_c[r][ch] + D_r X[r][c + ch C], ch = 16 b + (ln % 16)
            const int c = c0 + kc, ch0 = ln & 15;
            double z[NB];
            if constexpr (SPEC) {
#pragma unroll
              for (int b = 0; b < NB; ++b) z[b] = rv ? zval<true>(A, buf, d, n, with_p, c, r, 16 * b + ch0) : 0.0;
            } else {
              // unconditional reads (channel clamped into the sub-cube, rows
              // below S), so that they issue back to back; the select zeroes
              // rows past the segment and channels past L_c
              float xv[NB], pv[NB];
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                const int ch = min(16 * b + ch0, g.Lc - 1);
                xv[b] = buf[r * xrs + c + ch * g.C];
                pv[b] = with_p ? buf[pword(c, r, ch)] : 0.0f;
              }
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                const bool ok = rv && 16 * b + ch0 < g.Lc;
                const double zz = fma(dr, static_cast<double>(xv[b]), static_cast<double>(pv[b]));
                z[b] = ok ? zz : 0.0;
              }
            }
            int t = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
              for (int bj = bi; bj < NB; ++bj, ++t)
                acc[kc][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[bi], z[bj], acc[kc][t], 0, 0, 0);
          }
        }
      }
    }
  }
  drain_loads();
  // fixed-order sum of the four waves' partials, block pair by block pair
  double *red = reinterpret_cast<double *>(sm);
#pragma unroll
  for (int kc = 0; kc < K; ++kc) {
    if (kc < nc) {  // uniform
      int t = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj, ++t) {
          __syncthreads();
#pragma unroll
          for (int v = 0; v < 4; ++v) red[wave * 256 + v * 64 + ln] = static_cast<double>(acc[kc][t][v]);
          __syncthreads();
          const int e = threadIdx.x, v = e >> 6, l = e & 63;
          const double sum = red[e] + red[256 + e] + red[512 + e] + red[768 + e];
          // result layouts: v_mfma_f64_16x16x4f64 has lane l hold D[4 v + l / 16][l % 16],
          // v_mfma_f32_16x16x16_bf16 D[4 (l / 16) + v][l % 16]
          const int ii = 16 * bi + (BF16 ? 4 * (l / 16) + v : 4 * v + l / 16), jj = 16 * bj + (l & 15);
          const int f = (c0 + kc) * Q + q;
          A.gram[(static_cast<int64_t>(f) * A.chunks + chunk) * A.lc16 * A.lc16 + ii * A.lc16 + jj] = sum;
        }
    }
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

// One workgroup of kEigThreads per facet: each Jacobi round's row and column
// updates ((n/2) n elements each) spread over all its threads.
constexpr int kEigThreads = 1024;
constexpr int kEigSweeps = 40;

__global__ void __launch_bounds__(kEigThreads) nuc_eig_kernel(NucArgs A) {
  __shared__ double Am[kMaxLc][kMaxLc + 1];
  __shared__ double Vm[kMaxLc][kMaxLc + 1];
  __shared__ double cs_c[kMaxLc / 2], cs_s[kMaxLc / 2];
  __shared__ int cs_p[kMaxLc / 2], cs_q[kMaxLc / 2];
  __shared__ double lam[kMaxLc], hv[kMaxLc];
  __shared__ int rank[kMaxLc];
  __shared__ double red[kEigThreads / 64];
  const NucGeom &g = A.g;
  const int f = A.eig_q < 0 ? blockIdx.x : blockIdx.x * (g.qy * g.qx) + A.eig_q;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int n = g.Lc, n2 = n + (n & 1);
  if (A.sel != nullptr && A.sel[f] == 0) return;  // randomized step: facet not selected
  const FacetView F = facet_view(g, f);
  const int nch = (F.hy + A.chunk_wrows - 1) / A.chunk_wrows;
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
  for (int sweep = 0; sweep <= kEigSweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < n2 * n2; idx += nth) {
      const int i = idx / n2, j = idx - (idx / n2) * n2;
      const double a2 = Am[i][j] * Am[i][j];
      tot += a2;
      if (i != j) off += a2;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    // diagnostics: a Gram that is not finite (NaN or Inf in the input), or
    // off-diagonal energy still above 1e-20 of the total after the last sweep
    if (!(tot < __builtin_huge_val())) {
      if (tid == 0 && A.diag != nullptr) atomicAdd(A.diag + 1, 1u);
      break;
    }
    if (!(off > 1e-30 * tot)) break;
    if (sweep == kEigSweeps) {
      if (tid == 0 && A.diag != nullptr && off > 1e-20 * tot) atomicAdd(A.diag, 1u);
      break;
    }
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
    } else if (A.active == nullptr || A.active[F.c] != 0) {  // frozen sub-cubes keep theta_bar
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

// P_c <- Z_c K_c for every sub-cube, segment by segment (staging as in the
// Gram kernel).  Work items (sub-cube, 16-row block, 16-channel block) are
// spread over the waves; each is NB * 4 FP64 MFMAs with K_c read from LDS.
// The result goes to an LDS tile first and then to HBM as contiguous runs.
template <int NB, bool SPEC = false>
__global__ void __launch_bounds__(256) nuc_recon_kernel(NucArgs A) {
  constexpr int W = NB * 16;
  extern __shared__ float sm[];
  __shared__ double dsh[2][kMaxSeg];
  const NucGeom &g = A.g;
  const int q = A.q0 + blockIdx.y, chunk = blockIdx.x, Q = g.qy * g.qx;
  const FacetView F = facet_view(g, q);
  const int y0 = chunk * A.chunk_wrows;
  if (y0 >= F.hy) return;
  const int y1 = min(y0 + A.chunk_wrows, F.hy);
  const int S = A.seg, L = g.L, Lc = g.Lc, C = g.C;
  const int nsx = (F.hx + S - 1) / S, nseg = (y1 - y0) * nsx;
  const int BUF = stage_words(g, S);
  // LDS: K_c [C][W][W + 1] doubles, then two staging buffers, then the output tile [C][S][Lc]
  double *Ks = reinterpret_cast<double *>(sm);
  float *stage = sm + 2 * C * W * (W + 1);
  float *outt = stage + 2 * BUF;
  for (int idx = threadIdx.x; idx < C * W * W; idx += blockDim.x) {
    const int c = idx / (W * W), r = idx - c * W * W, i = r / W, j = r - (r / W) * W;
    Ks[(c * W + i) * (W + 1) + j] = A.kmat[static_cast<int64_t>(c * Q + q) * A.lc16 * A.lc16 + i * A.lc16 + j];
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  const int nrb = S / 16, ntask = C * nrb;

  issue_seg(A, F, seg_of(0, y0, nsx, S, F.hx), stage, dsh[0], true);
  for (int i = 0; i < nseg; ++i) {
    wait_loads_and_sync();
    if (i + 1 < nseg) issue_seg(A, F, seg_of(i + 1, y0, nsx, S, F.hx), stage + ((i + 1) & 1) * BUF, dsh[(i + 1) & 1], true);
    const float *buf = stage + (i & 1) * BUF;
    const double *d = dsh[i & 1];
    const Seg sg = seg_of(i, y0, nsx, S, F.hx);
    // tasks: (sub-cube, 16-row block) with Z's W / 4 slices formed once for
    // every 16-channel output block; when there are fewer such tasks than
    // waves, (sub-cube, row block, channel block) so that every wave works
    const bool split = ntask < 4;
    const int ntk = split ? ntask * NB : ntask;
    for (int t = wave; t < ntk; t += 4) {
      const int tt = split ? t / NB : t;
      const int c = tt / nrb, nb = tt - c * nrb;
      const int mb0 = split ? t - tt * NB : 0, mb1 = split ? mb0 + 1 : NB;
      const int r = 16 * nb + (ln & 15);
      double z[W / 4];
#pragma unroll
      for (int kk = 0; kk < W / 4; ++kk) z[kk] = zval<SPEC>(A, buf, d, sg.n, true, c, r, 4 * kk + ln / 16);
#pragma unroll
      for (int mb = 0; mb < NB; ++mb) {
        if (mb < mb0 || mb >= mb1) continue;
        v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < W / 4; ++kk) {
          const int k = 4 * kk + ln / 16;
          // A[m][k] = K[k][m], B[k][n] = Z[n][k]  ->  D[m][n] = (Z K)[n][m]
          const double a = Ks[(c * W + k) * (W + 1) + 16 * mb + (ln & 15)];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, z[kk], acc, 0, 0, 0);
        }
        if (r < sg.n) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = 16 * mb + 4 * v + ln / 16;
            if (m < Lc) outt[(c * S + r) * Lc + m] = static_cast<float>(acc[v]);
          }
        }
      }
    }
    __syncthreads();
    // contiguous runs of S x L_c floats per sub-cube, written in place into P
    const int nfl = sg.n * Lc;
    for (int c = 0; c < C; ++c) {
      if (A.active != nullptr && A.active[c] == 0) continue;  // a frozen sub-cube keeps its P
      if (A.sel != nullptr && A.sel[c * Q + q] == 0) continue;  // an unselected facet keeps its P
      float *dst = A.p + c * g.p_sub + F.poff + (static_cast<int64_t>(sg.y) * F.hx + sg.s0) * Lc;
      for (int e = threadIdx.x; e < nfl; e += blockDim.x) dst[e] = outt[c * S * Lc + e];
    }
  }
  drain_loads();
}

// One sub-cube (C = 1): each wave holds all of K (W x W) in registers and
// takes whole 16-row blocks of the segment (wave w: blocks w, w + 4, ...): it
// forms the block's Z once (16 rows x W channels, FP64) and runs the NB output
// channel blocks as NB interleaved MFMA accumulation chains, so LDS is read
// once per Z element and no wave waits on a single dependent chain.

template <int NB>
__global__ void __launch_bounds__(256) nuc_recon1_kernel(NucArgs A) {
  constexpr int W = NB * 16;
  constexpr int MAXRB = kMaxSeg / 16;  // row blocks per segment, upper bound
  extern __shared__ float sm[];
  __shared__ double dsh[2][kMaxSeg];
  const NucGeom &g = A.g;
  const int q = A.q0 + blockIdx.y, chunk = blockIdx.x;
  const FacetView F = facet_view(g, q);
  const int y0 = chunk * A.chunk_wrows;
  if (y0 >= F.hy) return;
  const int y1 = min(y0 + A.chunk_wrows, F.hy);
  if (A.active != nullptr && A.active[0] == 0) return;  // the one sub-cube is frozen: P stays
  if (A.sel != nullptr && A.sel[q] == 0) return;        // an unselected facet keeps its P
  const int S = A.seg, L = g.L, Lc = g.Lc;
  const int nsx = (F.hx + S - 1) / S, nseg = (y1 - y0) * nsx;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  const int nrb = S / 16;
  // kr[mb][kk] = K[4 kk + lane / 16][16 mb + lane % 16]: the B operand of
  // output channel block mb, contraction slice kk
  double kr[NB][W / 4];
  const double *Kq = A.kmat + static_cast<int64_t>(q) * A.lc16 * A.lc16;
#pragma unroll
  for (int mb = 0; mb < NB; ++mb)
#pragma unroll
    for (int kk = 0; kk < W / 4; ++kk) kr[mb][kk] = Kq[(4 * kk + ln / 16) * A.lc16 + 16 * mb + (ln & 15)];

  // staging: the padded 16-byte path (OneStage) when L is a multiple of 4,
  // else rows of L floats (X, then P at S L)
  const bool vec = L % 4 == 0;
  OneStage st;
  st.init(S, L, wave, ln);
  const int preg = vec ? st.preg : S * L;
  const int BUF = 2 * preg;
  const int rs = vec ? st.Lp : L;
  auto issue = [&](const Seg &sg, float *buf, double *dd) __attribute__((always_inline)) {
    if (vec)
      st.issue(A, F, sg, buf, dd, true, wave);
    else
      issue_seg(A, F, sg, buf, dd, true);
  };

  issue(seg_of(0, y0, nsx, S, F.hx), sm, dsh[0]);
  for (int i = 0; i < nseg; ++i) {
    wait_loads_and_sync();
    if (i + 1 < nseg) issue(seg_of(i + 1, y0, nsx, S, F.hx), sm + ((i + 1) & 1) * BUF, dsh[(i + 1) & 1]);
    float *buf = sm + (i & 1) * BUF;
    const double *d = dsh[i & 1];
    const Seg sg = seg_of(i, y0, nsx, S, F.hx);
    // results go straight from registers to P (rows of other segments are
    // never touched), so the stores drain while later row blocks compute
    float *dst = A.p + F.poff + (static_cast<int64_t>(sg.y) * F.hx + sg.s0) * Lc;
#pragma unroll 1
    for (int j = 0; j < MAXRB; j += 4) {
      const int nb = wave + j;
      if (nb < nrb) {
        const int r = 16 * nb + (ln & 15);
        // Z[r][k] = P[r][k] + D_r X[r][k] (one sub-cube: X and P rows have the
        // same layout), read at compile-time offsets from per-row bases; the
        // reads are unconditional (every address lies inside the staging
        // allocation, which has 64 words of slack past the last buffer) and a
        // select zeroes rows past the segment and channels past L_c
        const bool rv = r < sg.n;
        const float *xr = buf + r * rs + ln / 16, *pr = xr + preg;
        const double dr = d[r];
        double z[W / 4];
#pragma unroll
        for (int kk = 0; kk < W / 4; ++kk) {
          const double zz = fma(dr, static_cast<double>(xr[4 * kk]), static_cast<double>(pr[4 * kk]));
          z[kk] = (rv && 4 * kk + ln / 16 < Lc) ? zz : 0.0;
        }
        v4d res[NB];
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) res[mb] = v4d{0.0, 0.0, 0.0, 0.0};
        // A[n][k] = Z[n][k], B[k][m] = K[k][m]  ->  D[n][m] = (Z K)[n][m]
#pragma unroll
        for (int kk = 0; kk < W / 4; ++kk)
#pragma unroll
          for (int mb = 0; mb < NB; ++mb) res[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[kk], kr[mb][kk], res[mb], 0, 0, 0);
        // lane l holds D[4 v + l / 16][l % 16]: each store writes four rows of
        // 16 consecutive channels
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) {
          const int m = 16 * mb + (ln & 15);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rr = 16 * nb + 4 * v + ln / 16;
            if (rr < sg.n && m < Lc) dst[rr * Lc + m] = static_cast<float>(res[mb][v]);
          }
        }
      }
    }
  }
  drain_loads();
}

// A workgroup owns a run of kGatherPx pixels of one image row.  Its first
// threads resolve, once per pixel, the (at most four) covering facets: window
// weight and the offset of the pixel's row in each facet's P (sub-cube 0).
// Then thread t works on channel t % L of pixels t / L, t / L + 256 / L, ...:
// every P read and the gradient update are coalesced across the channels.
// SPEC (overlapping spectral facets): channel ch is column ch - (c sb - so)
// of its block c and, when it lies in the next block's leading so channels,
// of that block too, each weighted by its spectral ramp.
constexpr int kGatherPx = 256;

template <bool SPEC>
__global__ void __launch_bounds__(256) nuc_gather_kernel(GatherArgs A) {
  __shared__ double dk[kGatherPx][4];
  __shared__ int64_t rk[kGatherPx][4];
  const NucGeom &g = A.g;
  const int y = A.y_begin + blockIdx.y, x0 = A.x_begin + blockIdx.x * kGatherPx;
  const int npx = min(kGatherPx, A.x_end - x0);
  if (threadIdx.x < kGatherPx) {
    const int i = threadIdx.x, x = x0 + i;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      dk[i][k] = 0.0;
      rk[i][k] = 0;
    }
    if (i < npx) {
      const int sy0 = static_cast<int>((static_cast<int64_t>(y + 1) * g.qy + g.ny - 1) / g.ny) - 1;
      const int sx0 = static_cast<int>((static_cast<int64_t>(x + 1) * g.qx + g.nx - 1) / g.nx) - 1;
      const int ncy = (sy0 + 1 < g.qy && y >= g.ty[sy0 + 1] - g.oy) ? 2 : 1;
      const int ncx = (sx0 + 1 < g.qx && x >= g.tx[sx0 + 1] - g.ox) ? 2 : 1;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int dy = k >> 1, dx = k & 1;
        if (dy < ncy && dx < ncx) {
          const FacetView F = facet_view(g, (sy0 + dy) * g.qx + (sx0 + dx));
          const int yy = y - F.wy0, xx = x - F.wx0;
          dk[i][k] = ramp(yy, F.sy, g.qy, g.oy, F.hy) * ramp(xx, F.sx, g.qx, g.ox, F.hx);
          rk[i][k] = F.poff + (static_cast<int64_t>(yy) * F.hx + xx) * g.Lc;
        }
      }
    }
  }
  __syncthreads();
  const int L = g.L, per = 256 / L;  // pixels per pass of the workgroup (L <= 256)
  const int t = threadIdx.x;
  if (t >= per * L) return;
  const int ch = t % L;
  const float *pc, *pc2 = nullptr;
  double w1 = 1.0, w2 = 0.0;
  if constexpr (SPEC) {
    const int c1 = min(ch / g.sb, g.C - 1), col1 = ch - spec_chan(g, c1, 0);
    pc = A.p + c1 * g.p_sub + col1;
    w1 = spec_weight(g, c1, col1);
    if (c1 + 1 < g.C && ch >= spec_chan(g, c1 + 1, 0)) {
      const int col2 = ch - spec_chan(g, c1 + 1, 0);
      pc2 = A.p + (c1 + 1) * g.p_sub + col2;
      w2 = spec_weight(g, c1 + 1, col2);
    }
  } else {
    const int c = ch % g.C, l = ch / g.C;
    pc = A.p + c * g.p_sub + l;
  }
  float *grow = A.grad + (static_cast<int64_t>(y) * g.nx + x0) * L + ch;
  // U pixels per thread in flight: all their loads are issued before the first use
  constexpr int U = 4;
  for (int i0 = t / L; i0 < npx; i0 += U * per) {
    float pv[U][4], pv2[U][4], gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * per;
      const bool ok = i < npx;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool cov = ok && dk[ok ? i : 0][k] != 0.0;
        pv[u][k] = cov ? pc[rk[i][k]] : 0.0f;
        pv2[u][k] = (SPEC && cov && pc2 != nullptr) ? pc2[rk[i][k]] : 0.0f;
      }
      gv[u] = (ok && A.beta != 0.0f) ? grow[static_cast<int64_t>(i) * L] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * per;
      if (i < npx) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if constexpr (SPEC)
            sum += dk[i][k] * (w1 * static_cast<double>(pv[u][k]) + w2 * static_cast<double>(pv2[u][k]));
          else
            sum += dk[i][k] * static_cast<double>(pv[u][k]);
        }
        const float v = static_cast<float>(A.zeta * sum);
        grow[static_cast<int64_t>(i) * L] = A.beta != 0.0f ? fmaf(A.beta, gv[u], v) : v;
      }
    }
  }
}

static int check_launch(const char *what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string(what) + ": " + hipGetErrorString(err));
  return FHS_OK;
}

// dynamic LDS bytes of the Gram / reconstruction kernels
size_t nuc_lds_bytes(const NucArgs &a, bool recon) {
  const int W = a.lc16;
  // (+64 words: masked-out lanes read up to 63 words past a buffer)
  const size_t pw = static_cast<size_t>(a.g.C) * a.g.Lc;  // P floats per pixel over the sub-cubes
  const size_t stage = (2 * static_cast<size_t>(a.seg) * (a.g.L + pw) + 64) * sizeof(float);
  if (!recon) {
    const size_t gs =
        gram_one_stage(a.g) ? (2 * 2 * static_cast<size_t>(one_region(a.seg, a.g.L)) + 64) * sizeof(float) : stage;
    return gs > 8192 ? gs : 8192;  // the unit reduction reuses it (4 x 256 doubles)
  }
  return static_cast<size_t>(a.g.C) * W * (W + 1) * sizeof(double) + stage +
         static_cast<size_t>(a.seg) * pw * sizeof(float);
}

int launch_nuc_gram(const NucArgs &a, int nspatial, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t lds = nuc_lds_bytes(a, false);
#define FHS_GRAM_CASE(NB)                                                                               \
  case NB: {                                                                                            \
    constexpr int KM = gram_subcubes<NB>();                                                             \
    if (a.bf16) {                                                                                       \
      if (a.g.C == 1 || KM == 1)                                                                        \
        hipLaunchKernelGGL((nuc_gram_kernel<NB, 1, true>), dim3(a.chunks, nspatial, a.g.C), dim3(256), lds, s, a); \
      else                                                                                              \
        hipLaunchKernelGGL((nuc_gram_kernel<NB, KM, true>), dim3(a.chunks, nspatial, (a.g.C + KM - 1) / KM), \
                           dim3(256), lds, s, a);                                                       \
    } else if (a.g.spec) {                                                                              \
      if (KM == 1)                                                                                      \
        hipLaunchKernelGGL((nuc_gram_kernel<NB, 1, false, true>), dim3(a.chunks, nspatial, a.g.C), dim3(256), lds, s, \
                           a);                                                                          \
      else                                                                                              \
        hipLaunchKernelGGL((nuc_gram_kernel<NB, KM, false, true>),                                      \
                           dim3(a.chunks, nspatial, (a.g.C + KM - 1) / KM), dim3(256), lds, s, a);      \
    } else if (a.g.C == 1 || KM == 1) {                                                                 \
      hipLaunchKernelGGL((nuc_gram_kernel<NB, 1, false>), dim3(a.chunks, nspatial, a.g.C), dim3(256), lds, s, a); \
    } else {                                                                                            \
      hipLaunchKernelGGL((nuc_gram_kernel<NB, KM, false>), dim3(a.chunks, nspatial, (a.g.C + KM - 1) / KM), \
                         dim3(256), lds, s, a);                                                         \
    }                                                                                                   \
  } break;
  switch (a.lc16 / 16) {
    FHS_GRAM_CASE(1)
    FHS_GRAM_CASE(2)
    FHS_GRAM_CASE(3)
    FHS_GRAM_CASE(4)
    default: return fail(FHS_EUNSUPPORTED, "more than 64 channels per sub-cube");
  }
#undef FHS_GRAM_CASE
  return check_launch("nuc_gram");
}

int launch_nuc_eig(const NucArgs &a, int nfacets, void *stream) {
  hipLaunchKernelGGL(nuc_eig_kernel, dim3(nfacets), dim3(kEigThreads), 0, static_cast<hipStream_t>(stream), a);
  return check_launch("nuc_eig");
}

int launch_nuc_recon(const NucArgs &a, int nspatial, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(a.chunks, nspatial);
  if (a.g.C == 1) {
    // (+64 words: masked-out lanes read up to 63 words past a buffer)
    const int preg = a.g.L % 4 == 0 ? one_region(a.seg, a.g.L) : a.seg * a.g.L;
    const size_t lds1 = static_cast<size_t>(2 * 2 * preg + 64) * sizeof(float);
    switch (a.lc16 / 16) {
      case 1: hipLaunchKernelGGL(nuc_recon1_kernel<1>, grid, dim3(256), lds1, s, a); break;
      case 2: hipLaunchKernelGGL(nuc_recon1_kernel<2>, grid, dim3(256), lds1, s, a); break;
      case 3: hipLaunchKernelGGL(nuc_recon1_kernel<3>, grid, dim3(256), lds1, s, a); break;
      case 4: hipLaunchKernelGGL(nuc_recon1_kernel<4>, grid, dim3(256), lds1, s, a); break;
      default: return fail(FHS_EUNSUPPORTED, "more than 64 channels per sub-cube");
    }
    return check_launch("nuc_recon");
  }
  const size_t lds = nuc_lds_bytes(a, true);
  if (lds > 160 * 1024) return fail(FHS_EUNSUPPORTED, "reconstruction tile exceeds the LDS");
  if (a.g.spec) {
    switch (a.lc16 / 16) {
      case 1: hipLaunchKernelGGL((nuc_recon_kernel<1, true>), grid, dim3(256), lds, s, a); break;
      case 2: hipLaunchKernelGGL((nuc_recon_kernel<2, true>), grid, dim3(256), lds, s, a); break;
      case 3: hipLaunchKernelGGL((nuc_recon_kernel<3, true>), grid, dim3(256), lds, s, a); break;
      case 4: hipLaunchKernelGGL((nuc_recon_kernel<4, true>), grid, dim3(256), lds, s, a); break;
      default: return fail(FHS_EUNSUPPORTED, "more than 64 channels per facet matrix");
    }
    return check_launch("nuc_recon");
  }
  switch (a.lc16 / 16) {
    case 1: hipLaunchKernelGGL(nuc_recon_kernel<1>, grid, dim3(256), lds, s, a); break;
    case 2: hipLaunchKernelGGL(nuc_recon_kernel<2>, grid, dim3(256), lds, s, a); break;
    case 3: hipLaunchKernelGGL(nuc_recon_kernel<3>, grid, dim3(256), lds, s, a); break;
    case 4: hipLaunchKernelGGL(nuc_recon_kernel<4>, grid, dim3(256), lds, s, a); break;
    default: return fail(FHS_EUNSUPPORTED, "more than 64 channels per sub-cube");
  }
  return check_launch("nuc_recon");
}

int launch_nuc_gather(const GatherArgs &a, void *stream) {
  if (a.g.L > 256) return fail(FHS_EUNSUPPORTED, "gather: more than 256 channels");
  const dim3 grid((a.x_end - a.x_begin + kGatherPx - 1) / kGatherPx, a.y_end - a.y_begin);
  if (a.g.spec)
    hipLaunchKernelGGL(nuc_gather_kernel<true>, grid, dim3(256), 0, static_cast<hipStream_t>(stream), a);
  else
    hipLaunchKernelGGL(nuc_gather_kernel<false>, grid, dim3(256), 0, static_cast<hipStream_t>(stream), a);
  return check_launch("nuc_gather");
}

}  // namespace fhs
