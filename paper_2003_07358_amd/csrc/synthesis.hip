// SARA synthesis Psi w for gfx950: the exact adjoint of the analysis (Sec.
// 2.3.1; Alg. 2 facet synthesis summed over facets and the kappa
// term of aggregation).
//
// One level of the adjoint: an output sample x = 2k + px receives
// sum_{i < L/2} f[2i + 1 - px] c[k + i], so a thread owning coefficient column k
// produces output columns 2k and 2k+1, and output rows 2k' and 2k'+1 come from
// coefficient rows k' .. k' + L/2 - 1, whose horizontal adjoints are kept in a
// per-thread register ring.
//
// Levels >= 2 run one basis per workgroup and write the low-low band of the
// level above into the workspace.  Level 1 runs a group of bases per
// workgroup and sums them (and the Dirac basis) into the image in a fixed
// order: deterministic, no atomics.
//
// Memory pipeline: coefficient rows are grouped into phases of P rows whose
// four band segments are copied HBM -> LDS by buffer loads with LDS
// destination one phase ahead (double-buffered LDS), one barrier per phase;
// the values read at the outputs (Dirac band, previous image) are loaded into
// registers one phase ahead.
#include <hip/hip_runtime.h>

#include "fhs_filters.h"
#include "fhs_internal.h"
#include "lds_stage.h"

// waves per SIMD targeted by a level-1 synthesis group of more than two bases
constexpr int kFinalWavesPerEU = 2;

namespace fhs {

namespace {

constexpr int kOobS = static_cast<int>(0x80000000u);  // buffer offset past any range: loads 0, stores dropped

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_s(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0), static_cast<int>(bytes),
                                           0x00020000);
}
__device__ __forceinline__ float ld_f32s(__amdgpu_buffer_rsrc_t r, int voff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
__device__ __forceinline__ void st_f32s(float v, __amdgpu_buffer_rsrc_t r, int voff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, 0, 0);
}
// Waits until at most n (0, 4, 8, 16) of this wave's vector-memory operations
// are outstanding (they complete in issue order).
__device__ __forceinline__ void wait_vm_but_s(int n) {
  if (n == 4)
    asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  else if (n == 8)
    asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
  else if (n == 16)
    asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
  else
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
// Workgroup barrier without a memory fence.
__device__ __forceinline__ void barrier_s() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Segment j of a phase = (row j / 4, band j % 4): copy it into dst + j * segp.
__device__ __forceinline__ void issue_band_rows(const SynBand &B, int k0, int nrows, int kx0, int segn, int segp,
                                                int L, float *dst) {
  const int64_t rowlen = static_cast<int64_t>(B.Kx) * L;
  const int64_t c0 = static_cast<int64_t>(kx0) * L;
  const int wv = wave_id(), nwv = full_wave_count();
  if (wv >= nwv) return;
#pragma unroll
  for (int band = 0; band < 4; ++band) {
    const float *src = band == 0 ? B.ll : band == 1 ? B.lh : band == 2 ? B.hl : B.hh;
    for (int row = 0; row < nrows; ++row) {
      const int j = 4 * row + band;
      if (j % nwv != wv) continue;
      const int k = k0 + row;
      const bool kv = k >= 0 && k < B.Ky;
      wave_copy_row(src + (kv ? static_cast<int64_t>(k) * rowlen : 0), rowlen, c0, segn, kv, dst + j * segp);
    }
  }
}

// Horizontal adjoint of one staged coefficient row (bands at buf + b * segp)
// for both output parities.
template <int NTAP>
__device__ __forceinline__ void xadj(const float *buf, int segp, int off, int L, float &lo0, float &lo1, float &hi0,
                                     float &hi1) {
  using T = Taps<NTAP>;
  constexpr int H = NTAP / 2;
  lo0 = lo1 = hi0 = hi1 = 0.0f;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float cll = buf[off + i * L];
    const float clh = buf[segp + off + i * L];
    const float chl = buf[2 * segp + off + i * L];
    const float chh = buf[3 * segp + off + i * L];
    // even output column (px = 0): taps 2i+1 ; odd (px = 1): taps 2i
    lo0 = fmaf(T::h[2 * i + 1], cll, fmaf(T::g[2 * i + 1], clh, lo0));
    lo1 = fmaf(T::h[2 * i], cll, fmaf(T::g[2 * i], clh, lo1));
    hi0 = fmaf(T::h[2 * i + 1], chl, fmaf(T::g[2 * i + 1], chh, hi0));
    hi1 = fmaf(T::h[2 * i], chl, fmaf(T::g[2 * i], chh, hi1));
  }
}

template <int NTAP>
struct Ring {
  float lo[2][NTAP / 2], hi[2][NTAP / 2];  // [output parity][coefficient row, oldest first]
};

template <int NTAP>
__device__ __forceinline__ void ring_zero(Ring<NTAP> &R) {
#pragma unroll
  for (int i = 0; i < NTAP / 2; ++i) R.lo[0][i] = R.lo[1][i] = R.hi[0][i] = R.hi[1][i] = 0.0f;
}

template <int NTAP>
__device__ __forceinline__ void ring_push(const float *buf, int segp, int off, int L, Ring<NTAP> &R) {
  constexpr int H = NTAP / 2;
#pragma unroll
  for (int i = 0; i + 1 < H; ++i) {
    R.lo[0][i] = R.lo[0][i + 1];
    R.lo[1][i] = R.lo[1][i + 1];
    R.hi[0][i] = R.hi[0][i + 1];
    R.hi[1][i] = R.hi[1][i + 1];
  }
  xadj<NTAP>(buf, segp, off, L, R.lo[0][H - 1], R.lo[1][H - 1], R.hi[0][H - 1], R.hi[1][H - 1]);
}

// Vertical adjoint: adds the 2 x 2 outputs (rows 2k', 2k'+1) of the ring.
template <int NTAP>
__device__ __forceinline__ void ring_out(const Ring<NTAP> &R, float acc[2][2]) {
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

// ---------------------------------------------------------------- levels >= 2

template <int NTAP, int P>
__device__ __forceinline__ void syn_basis(const SynArgs &A, const SynBand &B, int wg, float *smem) {
  constexpr int H = NTAP / 2;
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  int lane, grp;
  bool idle;
  seg_map(tid, Lcp, lane, grp, idle);
  // (segments past the tile's tk columns, possible with dense widths, work
  // on column 0 and store nothing)
  const int c = grp % C, kq = grp / C < A.tk ? grp / C : 0;
  const bool lv = !idle && lane < Lc && grp / C < A.tk;
  const int p = c * Lc + lane;
  const int strip = wg % B.strips, yb = wg / B.strips;
  const int kx0 = B.x_begin / 2 + strip * A.tk;
  const int y0 = B.y_begin + yb * A.ty;
  const int y1 = min(y0 + A.ty, B.y_end);
  const int segn = (A.tk + H - 1) * L;
  const int segp = round_up(segn, 64);
  const int ks = y0 / 2;
  const int nout = (y1 - 1) / 2 - ks + 1;
  const int nk = nout + H - 1;
  const int nph = (nk + P - 1) / P;
  const int off = kq * L + p;
  const int x = 2 * (kx0 + kq);

  // byte offsets of this lane's two output pixels in an output row run that
  // starts at column 2 kx0, or out of range
  int vx[2];
#pragma unroll
  for (int px = 0; px < 2; ++px)
    vx[px] = (lv && x + px >= B.x_begin && x + px < B.x_end) ? ((2 * kq + px) * L + p) * 4 : kOobS;
  auto run = [&](int y) __attribute__((always_inline)) {
    const bool yv = y >= y0 && y < y1;
    return rsrc_s(B.out + (yv ? (static_cast<int64_t>(y) * B.nx + 2 * kx0) * L : 0), yv ? 0x7fffffffu : 0u);
  };

  Ring<NTAP> R;
  ring_zero(R);
  issue_band_rows(B, ks, P, kx0, segn, segp, L, smem);
  for (int ph = 0; ph < nph; ++ph) {
    // the phase's copies precede the previous phase's 4P stores, a fixed
    // four per step (dropped outside the tile), the only later vector-memory
    // operations of this wave
    if (ph == 0)
      wait_vm_but_s(0);
    else
      wait_vm_but_s(4 * P);
    barrier_s();
    if (ph + 1 < nph) issue_band_rows(B, ks + (ph + 1) * P, P, kx0, segn, segp, L, smem + ((ph + 1) & 1) * 4 * P * segp);
    const float *buf = smem + (ph & 1) * 4 * P * segp;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int r = ph * P + k;
      if (r < nk) {
        ring_push<NTAP>(buf + 4 * k * segp, segp, off, L, R);
        if (r >= H - 1) {
          const int kp = ks + r - (H - 1);
          float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
          ring_out<NTAP>(R, acc);
#pragma unroll
          for (int py = 0; py < 2; ++py) {
            const __amdgpu_buffer_rsrc_t ro = run(2 * kp + py);
#pragma unroll
            for (int px = 0; px < 2; ++px) st_f32s(acc[py][px], ro, vx[px]);
          }
        } else {
          const __amdgpu_buffer_rsrc_t none = rsrc_s(B.out, 0u);
#pragma unroll
          for (int i = 0; i < 4; ++i) st_f32s(0.0f, none, kOobS + 1024 * i);
        }
      }
    }
  }
  drain_loads();
}

}  // namespace

template <int P>
__global__ void __launch_bounds__(FHS_SYN_THREADS) syn_kernel(SynArgs A) {
  extern __shared__ float smem[];
  const int id = blockIdx.x;
  int b = 0;
  while (b < kBases - 1 && id >= A.wg_prefix[b + 1]) ++b;
  const int wg = id - A.wg_prefix[b];
  switch (b) {
    case 0: syn_basis<2, P>(A, A.b[0], wg, smem); break;
    case 1: syn_basis<4, P>(A, A.b[1], wg, smem); break;
    case 2: syn_basis<6, P>(A, A.b[2], wg, smem); break;
    case 3: syn_basis<8, P>(A, A.b[3], wg, smem); break;
    case 4: syn_basis<10, P>(A, A.b[4], wg, smem); break;
    case 5: syn_basis<12, P>(A, A.b[5], wg, smem); break;
    case 6: syn_basis<14, P>(A, A.b[6], wg, smem); break;
    default: syn_basis<16, P>(A, A.b[7], wg, smem); break;
  }
}

static int syn_segp(int tk, int L) { return ((tk + kMaxTap / 2 - 1) * L + 63) / 64 * 64; }

int launch_synthesis(const SynArgs &a, int nthreads, void *stream) {
  const int nwg = a.wg_prefix[kBases];
  if (nwg <= 0) return FHS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int segp = syn_segp(a.tk, a.L);
  const int P = 2 * 4 * 4 * segp * 4 <= 65536 ? 4 : 2;
  const size_t lds = static_cast<size_t>(2 * 4 * P * segp) * sizeof(float);
  if (P == 4)
    hipLaunchKernelGGL(syn_kernel<4>, dim3(nwg), dim3(nthreads), lds, s, a);
  else
    hipLaunchKernelGGL(syn_kernel<2>, dim3(nwg), dim3(nthreads), lds, s, a);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("synthesis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

// ---------------------------------------------------------------- level 1

namespace {

// Bases [0, kFinalSplit) go in the first final-level pass, the rest in the second.
constexpr int kFinalSplit = 4;

// LDS floats of one staged band row of basis b.
__device__ __forceinline__ int fin_segp(int tk, int b, int L) { return round_up((tk + b) * L, 64); }

// The rings of bases b .. BEND-1 (basis b has 2(b+1) taps and b+1 rows per ring).
// At output step s basis b needs coefficient row ks + s + b, so it starts b
// steps before the first output.
template <int b, int BEND, int P>
struct RingSet {
  Ring<2 * (b + 1)> r;
  RingSet<b + 1, BEND, P> next;
  __device__ __forceinline__ void zero() {
    ring_zero(r);
    next.zero();
  }
  __device__ __forceinline__ void push(const SynFinalArgs &A, int s, int k, int off, int L, const float *lds) {
    const int segp = fin_segp(A.tk, b, L);
    if (s >= -b) ring_push<2 * (b + 1)>(lds + 4 * k * segp, segp, off, L, r);
    next.push(A, s, k, off, L, lds + 4 * P * segp);
  }
  __device__ __forceinline__ void out(float acc[2][2]) {
    ring_out<2 * (b + 1)>(r, acc);
    next.out(acc);
  }
};

template <int BEND, int P>
struct RingSet<BEND, BEND, P> {
  __device__ __forceinline__ void zero() {}
  __device__ __forceinline__ void push(const SynFinalArgs &, int, int, int, int, const float *) {}
  __device__ __forceinline__ void out(float[2][2]) {}
};

}  // namespace

// Bases B0 .. B1-1 of level 1 summed into the image; FIRST also adds the Dirac
// basis and applies beta, the second group accumulates onto the first.
//
// Vector-memory order per phase: the values read at the outputs of the next
// phase (loaded into registers), then the next phase's band copies, then the
// phase's output stores, a fixed four per step (range-checked buffer stores;
// out-of-range lanes and the steps before the first output store nothing).
// The wait at a phase boundary therefore leaves the previous phase's stores in
// flight, and the barrier carries no memory fence.
template <int B0, int B1, bool FIRST, int P>
__global__ void __launch_bounds__(FHS_SYN_THREADS)
__attribute__((amdgpu_waves_per_eu(B1 - B0 <= 2 ? 2 * kFinalWavesPerEU : kFinalWavesPerEU)))
syn_final_kernel(SynFinalArgs A) {
  extern __shared__ float smem[];
  const int L = A.L, Lcp = A.Lcp, C = A.C, Lc = A.Lc;
  const int tid = threadIdx.x;
  int lane, grp;
  bool idle;
  seg_map(tid, Lcp, lane, grp, idle);
  const int c = grp % C, kq = grp / C < A.tk ? grp / C : 0;
  const bool lv = !idle && lane < Lc && grp / C < A.tk;
  const int p = c * Lc + lane;
  const int ch = A.contig ? p : c + lane * C;  // natural channel order of the image
  const int strip = blockIdx.x % A.strips, yb = blockIdx.x / A.strips;
  const int kx0 = A.x_begin / 2 + strip * A.tk;
  const int y0 = A.y_begin + yb * A.ty;
  const int y1 = min(y0 + A.ty, A.y_end);
  const int ks = y0 / 2;
  const int nout = (y1 - 1) / 2 - ks + 1;
  const int x = 2 * (kx0 + kq);
  const int off = kq * L + p;
  int half = 0;  // floats of one phase buffer
  for (int b = B0; b < B1; ++b) half += 4 * P * fin_segp(A.tk, b, L);
  RingSet<B0, B1, P> R;
  R.zero();

  // Band-row copies: descriptors of the group's bands in LDS (read back as
  // wave-uniform values when a copy is issued, so that the 4 (B1 - B0) band
  // addresses do not occupy scalar registers across the loop), and the copy
  // work of a phase spread over the waves as (basis, row, band) tasks.
  constexpr int NB = B1 - B0;
  __shared__ uint64_t dsc_base[NB][4];       // byte address of row 0 at column kx0
  __shared__ uint32_t dsc_rec[NB], dsc_row[NB];  // bytes from column kx0 to the row end; bytes per row
  __shared__ int dsc_ky[NB], dsc_off[NB];    // rows; offset of the basis' region in a phase buffer (floats)
  if (tid < 4 * NB) {
#pragma unroll
    for (int bb = B0; bb < B1; ++bb)
      if ((tid >> 2) == bb - B0) {
        const SynBand &S = A.b[bb];
        const int band = tid & 3;
        const float *src = band == 0 ? S.ll : band == 1 ? S.lh : band == 2 ? S.hl : S.hh;
        dsc_base[bb - B0][band] = reinterpret_cast<uint64_t>(src + static_cast<int64_t>(kx0) * L);
        if (band == 0) {
          dsc_rec[bb - B0] = static_cast<uint32_t>(max(0, S.Kx - kx0)) * L * 4;
          dsc_row[bb - B0] = static_cast<uint32_t>(S.Kx) * L * 4;
          dsc_ky[bb - B0] = S.Ky;
          int o = 0;
          for (int b2 = B0; b2 < bb; ++b2) o += 4 * P * fin_segp(A.tk, b2, L);
          dsc_off[bb - B0] = o;
        }
      }
  }
  __syncthreads();
  const int wv = wave_id(), nwv = full_wave_count(), ln = tid & 63;
  auto issue = [&](int s0, float *lds) __attribute__((always_inline)) {
    for (int t = wv; t < NB * 4 * P && wv < nwv; t += nwv) {
      const int bi = t / (4 * P), rem = t - bi * 4 * P, row = rem >> 2, band = rem & 3;
      const int b = B0 + bi;
      const int k = ks + s0 + b + row;  // coefficient row
      const int ky = __builtin_amdgcn_readfirstlane(dsc_ky[bi]);
      const bool kv = k >= 0 && k < ky;
      const uint64_t base = dsc_base[bi][band];
      const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(base));
      const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(base >> 32));
      const uint32_t rowb = __builtin_amdgcn_readfirstlane(dsc_row[bi]);
      const uint32_t rec = __builtin_amdgcn_readfirstlane(dsc_rec[bi]);
      const char *rp = reinterpret_cast<const char *>((static_cast<uint64_t>(hi) << 32) | lo) +
                       (kv ? static_cast<uint64_t>(k) * rowb : 0);
      const fhs_int32x4 rs = buffer_rsrc(rp, kv ? rec : 0u);
      const int segn = (A.tk + b) * L, segp = round_up(segn, 64);
      float *dst = lds + __builtin_amdgcn_readfirstlane(dsc_off[bi]) + (4 * row + band) * segp;
      for (int j = 0; j < segn; j += 64)
        fhs_raw_buffer_load_lds(rs, lds_words(dst + j), 4, (j + ln) * 4, 0, 0, 0);
    }
  };
  const float scale = A.alpha * (1.0f / 3.0f);
  const int sfirst = -(B1 - 1);
  const int nsteps = nout - sfirst;
  const int nph = (nsteps + P - 1) / P;
  // byte offsets of this lane's two output pixels in an image row run that
  // starts at column 2 kx0 (natural order for the image, positions for the
  // Dirac band), or out of range
  int vx[2], vd[2];
#pragma unroll
  for (int px = 0; px < 2; ++px) {
    const bool in = lv && x + px >= A.x_begin && x + px < A.x_end;
    vx[px] = in ? ((2 * kq + px) * L + ch) * 4 : kOobS;
    vd[px] = in ? ((2 * kq + px) * L + p) * 4 : kOobS;
  }
  const int64_t row_floats = static_cast<int64_t>(A.nx) * L;
  // the image (or Dirac band) row run of output row y, empty outside the tile's rows
  auto run = [&](const float *base, int y) __attribute__((always_inline)) {
    const bool yv = y >= y0 && y < y1;
    return rsrc_s(base + (yv ? static_cast<int64_t>(y) * row_floats + static_cast<int64_t>(2 * kx0) * L : 0),
                  yv ? 0x7fffffffu : 0u);
  };

  // Fused Dirac-band dual update (first group, when xin is given): the
  // Dirac coefficient of an output pixel is updated here, W_d <- W_d + xin / 3
  // shrunk by its l2 row norm over the sub-cube's channels (the analysis'
  // Dirac arithmetic, operation for operation), stored, and enters the output.
  const bool fuse = FIRST && A.xin != nullptr;
  const float thr = fuse ? static_cast<float>(A.mu[c] * A.inv_kappa) : 0.0f;
  // a frozen sub-cube keeps its Dirac rows (the old value is stored back)
  const bool act = !fuse || A.active == nullptr || A.active[c] != 0;
  // theta word of this lane's two pixels in a row run starting at column 2 kx0
  int vt[2];
#pragma unroll
  for (int px = 0; px < 2; ++px)
    vt[px] = vd[px] != kOobS ? static_cast<int>((static_cast<int64_t>(c) * A.I + A.dirac_row + 2 * kx0 + 2 * kq + px) * 4)
                             : kOobS;
  // theta of output row y (empty outside the tile's rows); soffset: the row
  auto trow = [&](int y, int &so) __attribute__((always_inline)) {
    const bool yv = fuse && y >= y0 && y < y1;
    so = yv ? static_cast<int>(static_cast<int64_t>(y) * A.nx * 4) : 0;
    return rsrc_s(A.theta, yv ? static_cast<uint32_t>(A.theta_bytes) : 0u);
  };
  const int stores = fuse ? 8 : 4;  // per step, fixed (the phase wait counts them)

  // values read at the outputs of step s: the Dirac coefficient and beta's
  // previous image (first group; fused: also the analysis input and theta) or
  // the image of the first group (second)
  auto pre = [&](int s, float v[2][2], float gv[2][2], float xv[2][2], float tv[2][2]) __attribute__((always_inline)) {
#pragma unroll
    for (int py = 0; py < 2; ++py) {
      const int y = (s >= 0 && s < nout) ? 2 * (ks + s) + py : -1;
      const __amdgpu_buffer_rsrc_t rx = run(A.x, y);
      int so = 0;
      const __amdgpu_buffer_rsrc_t rt = trow(y, so);
#pragma unroll
      for (int px = 0; px < 2; ++px) {
        xv[py][px] = tv[py][px] = 0.0f;
        if (FIRST) {
          v[py][px] = ld_f32s(run(A.dirac, y), vd[px]);
          gv[py][px] = A.beta != 0.0f ? ld_f32s(rx, vx[px]) : 0.0f;
          if (fuse) {
            xv[py][px] = ld_f32s(run(A.xin, y), vx[px]);
            tv[py][px] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rt, vt[px], so, 0));
          }
        } else {
          v[py][px] = ld_f32s(rx, vx[px]);
          gv[py][px] = 0.0f;
        }
      }
    }
  };
  float vq[P][2][2], gq[P][2][2], xq[P][2][2], tq[P][2][2];
#pragma unroll
  for (int k = 0; k < P; ++k) pre(sfirst + k, vq[k], gq[k], xq[k], tq[k]);
  issue(sfirst, smem);

  for (int ph = 0; ph < nph; ++ph) {
    if (ph == 0)
      wait_vm_but_s(0);
    else
      wait_vm_but_s(stores * P);
    // (the compiler's own wait for the loaded output values: they were
    // issued before the copies just waited for)
#pragma unroll
    for (int k = 0; k < P; ++k) {
      asm volatile("" ::"v"(vq[k][0][0]), "v"(vq[k][0][1]), "v"(vq[k][1][0]), "v"(vq[k][1][1]), "v"(gq[k][0][0]),
                   "v"(gq[k][0][1]), "v"(gq[k][1][0]), "v"(gq[k][1][1]));
      asm volatile("" ::"v"(xq[k][0][0]), "v"(xq[k][0][1]), "v"(xq[k][1][0]), "v"(xq[k][1][1]), "v"(tq[k][0][0]),
                   "v"(tq[k][0][1]), "v"(tq[k][1][0]), "v"(tq[k][1][1]));
    }
    barrier_s();
    float vcur[P][2][2], gcur[P][2][2], xcur[P][2][2], tcur[P][2][2];
#pragma unroll
    for (int k = 0; k < P; ++k)
#pragma unroll
      for (int py = 0; py < 2; ++py)
#pragma unroll
        for (int px = 0; px < 2; ++px) {
          vcur[k][py][px] = vq[k][py][px];
          gcur[k][py][px] = gq[k][py][px];
          xcur[k][py][px] = xq[k][py][px];
          tcur[k][py][px] = tq[k][py][px];
        }
    if (ph + 1 < nph) {
#pragma unroll
      for (int k = 0; k < P; ++k) pre(sfirst + (ph + 1) * P + k, vq[k], gq[k], xq[k], tq[k]);
      issue(sfirst + (ph + 1) * P, smem + ((ph + 1) & 1) * half);
    }
    const float *buf = smem + (ph & 1) * half;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int s = sfirst + ph * P + k;
      if (s < nout) {
        R.push(A, s, k, off, L, buf);
        if (s >= 0) {
          float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
          R.out(acc);
          const int kp = ks + s;
#pragma unroll
          for (int py = 0; py < 2; ++py) {
            const __amdgpu_buffer_rsrc_t rx = run(A.x, 2 * kp + py);
            float wd[2] = {vcur[k][py][0], vcur[k][py][1]};
            if (fuse) {
              const __amdgpu_buffer_rsrc_t rd = run(A.dirac, 2 * kp + py);
#pragma unroll
              for (int px = 0; px < 2; ++px) {
                const float nw = l21_row_update(vcur[k][py][px], xcur[k][py][px], thr * tcur[k][py][px], Lcp);
                wd[px] = act ? nw : vcur[k][py][px];
                st_f32s(wd[px], rd, vd[px]);
              }
            }
#pragma unroll
            for (int px = 0; px < 2; ++px) {
              float o;
              if (FIRST) {
                const float v = scale * (acc[py][px] + wd[px]);
                o = A.beta != 0.0f ? fmaf(A.beta, gcur[k][py][px], v) : v;
              } else {
                o = fmaf(scale, acc[py][px], vcur[k][py][px]);
              }
              st_f32s(o, rx, vx[px]);
            }
          }
        } else {
          // (steps before the first output: dropped stores at distinct,
          // non-adjacent offsets, which the compiler cannot merge)
          const __amdgpu_buffer_rsrc_t none = rsrc_s(A.x, 0u);
#pragma unroll
          for (int i = 0; i < 4; ++i) st_f32s(0.0f, none, kOobS + 1024 * i);
          if (fuse)
#pragma unroll
            for (int i = 4; i < 8; ++i) st_f32s(0.0f, none, kOobS + 1024 * i);
        }
      }
    }
  }
  drain_loads();
}

static int final_half_floats(int tk, int L, int b0, int b1, int P) {
  int half = 0;
  for (int b = b0; b < b1; ++b) half += 4 * P * (((tk + b) * L + 63) / 64 * 64);
  return half;
}

template <int B0, int B1, bool FIRST>
static void launch_final_group(const SynFinalArgs &a, int nthreads, hipStream_t s) {
  const int nwg = a.strips * a.yblocks;
  const int P = 2 * final_half_floats(a.tk, a.L, B0, B1, 2) * 4 <= 65536 ? 2 : 1;
  const size_t lds = static_cast<size_t>(2 * final_half_floats(a.tk, a.L, B0, B1, P)) * sizeof(float);
  if (P == 2)
    hipLaunchKernelGGL((syn_final_kernel<B0, B1, FIRST, 2>), dim3(nwg), dim3(nthreads), lds, s, a);
  else
    hipLaunchKernelGGL((syn_final_kernel<B0, B1, FIRST, 1>), dim3(nwg), dim3(nthreads), lds, s, a);
}

// group 0: bases [0, kFinalSplit) + Dirac (applies beta); groups 1 and 2:
// the rest in two halves (fewer rings per thread: more waves per SIMD).
int launch_synthesis_final(const SynFinalArgs &a, int nthreads, int group, void *stream) {
  if (a.strips * a.yblocks <= 0) return FHS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  constexpr int kMid = (kFinalSplit + kBases) / 2;
  if (group == 0)
    launch_final_group<0, kFinalSplit, true>(a, nthreads, s);
  else if (group == 1)
    launch_final_group<kFinalSplit, kMid, false>(a, nthreads, s);
  else
    launch_final_group<kMid, kBases, false>(a, nthreads, s);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(FHS_EHIP, std::string("final synthesis launch: ") + hipGetErrorString(err));
  return FHS_OK;
}

}  // namespace fhs
