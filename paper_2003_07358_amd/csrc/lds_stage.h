// Device helpers shared by the wavelet kernels: staging contiguous HBM
// segments into LDS with buffer loads whose destination is LDS, and the
// channel-segment reduction used by the l21 row norm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

typedef int fhs_int32x4 __attribute__((ext_vector_type(4)));

// Buffer load whose data goes to LDS: lane i of the wave writes `size` bytes at
// lds + i * size (lds must be wave-uniform).  Out-of-range offsets (buffer range
// checking) write zeros.
__device__ void fhs_raw_buffer_load_lds(fhs_int32x4 rsrc, __attribute__((address_space(3))) unsigned int *lds,
                                        int size, int voffset, int soffset, int offset,
                                        int aux) __asm("llvm.amdgcn.raw.buffer.load.lds");

namespace fhs {

__device__ __forceinline__ fhs_int32x4 buffer_rsrc(const void *base, unsigned bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  fhs_int32x4 r;
  r.x = static_cast<int>(a & 0xffffffffu);
  r.y = static_cast<int>((a >> 32) & 0xffffu);  // stride 0
  r.z = static_cast<int>(bytes);                 // range in bytes
  r.w = 0x00020000;                              // gfx9-family raw-buffer word 3
  return r;
}

__device__ __forceinline__ int round_up(int n, int m) { return (n + m - 1) / m * m; }

__device__ __forceinline__ __attribute__((address_space(3))) unsigned int *lds_words(const float *p) {
  return reinterpret_cast<__attribute__((address_space(3))) unsigned int *>(reinterpret_cast<uintptr_t>(p));
}

// The full waves of the workgroup copy floats [0, n) of src into dst (LDS),
// 64-float chunks spread over the waves; lanes past n do not write.
__device__ __forceinline__ void copy_span(const float *src, int n, float *dst) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwv = blockDim.x >> 6;
  if (wv >= nwv || n <= 0) return;
  const fhs_int32x4 rsrc = buffer_rsrc(src, static_cast<unsigned>(n) * 4u);
  const int ln = threadIdx.x & 63;
  for (int j = wv * 64; j < n; j += nwv * 64)
    if (j + ln < n) fhs_raw_buffer_load_lds(rsrc, lds_words(dst + j), 4, (j + ln) * 4, 0, 0, 0);
}

// One wave copies floats [seg0, seg0 + n) of `row` (zero outside [0, rowlen),
// or everywhere when !valid) into dst[0 .. n); dst must hold round_up(n, 64)
// floats (the lanes past n write zeros there).
__device__ __forceinline__ void wave_copy_row(const float *row, int64_t rowlen, int64_t seg0, int n, bool valid,
                                              float *dst) {
  const fhs_int32x4 rsrc = buffer_rsrc(row, valid ? static_cast<unsigned>(rowlen * 4) : 0u);
  const int lane = threadIdx.x & 63;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    const int64_t gi = seg0 + i;
    const int voff = (i < n && gi >= 0 && gi < rowlen) ? static_cast<int>(gi * 4) : static_cast<int>(0x80000000u);
    __attribute__((address_space(3))) unsigned int *l =
        reinterpret_cast<__attribute__((address_space(3))) unsigned int *>(reinterpret_cast<uintptr_t>(dst + base));
    fhs_raw_buffer_load_lds(rsrc, l, 4, voff, 0, 0, 0);
  }
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
// Waves with all 64 lanes present: only these issue LDS copies (a partial wave
// would leave the slots of its missing lanes unwritten).  The launchers use
// at least 64 threads per workgroup.
__device__ __forceinline__ int full_wave_count() { return blockDim.x >> 6; }

// All of this thread's outstanding vector-memory operations complete (the
// LDS copies included), then a workgroup barrier.
__device__ __forceinline__ void wait_loads_and_sync() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

__device__ __forceinline__ void drain_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Sum over the segment of `lcp` lanes holding this lane, every lane of the
// segment receiving the sum (dense widths: see seg_sum).  Power-of-two widths
// (aligned segments): a butterfly whose cross-lane moves all stay in the VALU:
// DPP quad permutations (lane ^ 1, lane ^ 2), DPP half-row and row mirrors
// (which pair the two halves of 8 and of 16 lanes), then the gfx950 row swaps:
// v_permlane16_swap of a value with itself leaves rows (0, 0, 2, 2) in one
// result and (1, 1, 3, 3) in the other, so their sum is the 32-lane pair sum
// in every lane; v_permlane32_swap does the same for the two halves of the
// wave.  (Addition is commutative bit for bit, so every lane of a segment
// gets the same sum.)
// (update_dpp with bound_ctrl lets the compiler fold the move into the add:
// one v_add_f32 with a DPP source)
__device__ __forceinline__ float dpp_add(float v, int ctrl_tag) {
  int o;
  const int iv = __float_as_int(v);
  switch (ctrl_tag) {
    case 0: o = __builtin_amdgcn_update_dpp(0, iv, 0xB1, 0xF, 0xF, true); break;   // quad [1,0,3,2]
    case 1: o = __builtin_amdgcn_update_dpp(0, iv, 0x4E, 0xF, 0xF, true); break;   // quad [2,3,0,1]
    case 2: o = __builtin_amdgcn_update_dpp(0, iv, 0x141, 0xF, 0xF, true); break;  // row half mirror
    default: o = __builtin_amdgcn_update_dpp(0, iv, 0x140, 0xF, 0xF, true); break; // row mirror
  }
  return v + __int_as_float(o);
}

// Lane segments.  A power-of-two width lcp tiles the workgroup (thread t is
// lane t % lcp of segment t / lcp).  The dense widths (6, 10, 12, 18, 20: even,
// not a power of two) tile each wave with 64 / lcp whole segments, the
// remaining 64 mod lcp lanes of the wave being idle: they alias lane 0 of the
// wave's first segment (so every address they form is a valid one) and must
// store nothing.
__device__ __forceinline__ constexpr bool dense_width(int lcp) { return (lcp & (lcp - 1)) != 0; }

__device__ __forceinline__ void seg_map(int tid, int lcp, int &lane, int &seg, bool &idle) {
  if (!dense_width(lcp)) {
    lane = tid % lcp;
    seg = tid / lcp;
    idle = false;
  } else {
    const int ln = tid & 63, g = 64 / lcp;
    idle = ln >= g * lcp;
    lane = idle ? 0 : ln % lcp;
    seg = (tid >> 6) * g + (idle ? 0 : ln / lcp);
  }
}

// Whole segments of a dense width per workgroup of `threads` threads.
__host__ __device__ __forceinline__ int dense_segments(int threads, int lcp) { return (threads / 64) * (64 / lcp); }

__device__ __forceinline__ float seg_sum(float v, int lcp) {
  if (dense_width(lcp)) {
    // pair (or, for a multiple of 4, quad) sums, every lane of a pair / quad
    // getting the same bits, then the segment's pair / quad sums fetched and
    // added in one fixed order
    const int grain = lcp % 4 == 0 ? 4 : 2;
    v = dpp_add(v, 0);
    if (grain == 4) v = dpp_add(v, 1);
    const int base = ((threadIdx.x & 63) / lcp) * lcp * 4;
    const int iv = __float_as_int(v);
    float s = __int_as_float(__builtin_amdgcn_ds_bpermute(base, iv));
    for (int j = 1; j < lcp / grain; ++j) s += __int_as_float(__builtin_amdgcn_ds_bpermute(base + 4 * grain * j, iv));
    return s;
  }
  if (lcp >= 2) v = dpp_add(v, 0);
  if (lcp >= 4) v = dpp_add(v, 1);
  if (lcp >= 8) v = dpp_add(v, 2);
  if (lcp >= 16) v = dpp_add(v, 3);
  if (lcp >= 32) {
    const unsigned u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  if (lcp >= 64) {
    const unsigned u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  return v;
}

// The l21 row update of one coefficient held by a lane of an lcp-lane segment
// (the segment holds the row over a sub-cube's channels): u = w + v/3, then
// u min(1, thr_th / ||u||). Products are never contracted into the adds, so
// that every kernel applying it (the analysis' Dirac pass and the level-1
// synthesis that fuses it) produces the same bits.
__device__ __forceinline__ float l21_row_update(float w, float v, float thr_th, int lcp) {
#pragma clang fp contract(off)
  const float u = w + v * (1.0f / 3.0f);
  const float r2 = seg_sum(u * u, lcp);
  return u * fminf(1.0f, thr_th * __frsqrt_rn(r2));
}

}  // namespace fhs
