// Internal declarations of the data-fidelity block (measurement operator and
// the data dual update): the data plan and the kernel launchers.
#pragma once

#include <cstdint>
#include <vector>

#include "fhs.h"

namespace fhs {
namespace data {

constexpr int kKbWidth = 7;      // Kaiser-Bessel kernel width J (7 x 7 de-gridding)
constexpr int kOversample = 2;   // grid points per image pixel and axis
constexpr int kMaxGrid = 8192;   // largest grid axis (one FFT row in LDS)
constexpr int kDualThreads = 256;
constexpr int kDualBlocks = 128; // workgroups per channel of the data dual passes
constexpr int kGridTile = 32;    // gridding: grid points per tile side (LDS accumulation)
constexpr int kGridChunk = 2048; // gridding: visibilities per work item

struct float2v {
  float x, y;
};

// Per-visibility interpolation entry: channel, first grid index on each axis
// (already reduced modulo the grid size).
struct VisInfo {
  int32_t chan, k1, k2, pad;
};

// Gridding work item: the visibilities perm[start .. start + count) of channel
// chan whose first grid indices lie in tile (t1, t2) of kGridTile points.
struct GridItem {
  int32_t chan, t1, t2, start, count, pad0, pad1, pad2;
};

// Arguments of the launchers (device pointers into the workspace / caller arrays).
struct PadArgs {
  const float *x;          // [ny][nx][L]
  float2v *grid;           // [L][K1][K2]
  const float *s1, *s2;    // [ny], [nx] scaling of Z
  int ny, nx, L, K1, K2;
};

struct CropArgs {
  const float2v *grid;     // [L][K1][K2]
  float *x;                // [ny][nx][L]
  const float *s1, *s2;
  const double *scale;     // [L] or null (1)
  float beta;
  int ny, nx, L, K1, K2;
};

struct InterpArgs {
  const float2v *spec;     // [L][K2][K1] (the transposed spectrum)
  float2v *grid;           // adjoint target, same layout
  const float2v *vis_in;   // adjoint input
  float2v *vis_out;        // forward output
  const VisInfo *info;     // [M]
  const float *w;          // [M][2 J]: the J weights of axis 1, then of axis 2
  const int32_t *perm;     // gridding: visibilities sorted by (channel, tile)
  const GridItem *items;   // gridding work items
  int64_t m, n_items;
  int K1, K2;
  int wexp;                // gridding: every product of two weights is below 2^wexp
};

struct DualArgs {
  const float2v *yc;       // Phi xcheck  [M]
  const float2v *yx;       // Phi x       [M]
  float2v *v;              // in / out    [M]
  const float2v *y;        // data        [M]
  const float *U;          // [M] diagonal preconditioner (> 0)
  float2v *p;              // [M] workspace: the projection iterate
  const double *eps;       // [L] l2-ball radii
  const int64_t *voff;     // [L + 1] first visibility of each channel
  double *residual;        // [L] ||y - Phi x|| or null
  double *part;            // [L][kDualBlocks][4] workgroup partial sums (workspace)
  double *chs;             // [L][4] per channel: ball factor, gamma, residual (workspace)
  int n_sub;
  int L;
};

int launch_pad(const PadArgs &a, void *stream);
int launch_crop(const CropArgs &a, void *stream);
int launch_fft_rows(float2v *data, int64_t rows, int K, const float2v *tw, int sign, void *stream);
int launch_transpose(const float2v *in, float2v *out, int R, int Cc, int planes, void *stream);
int launch_fill_zero(float2v *data, int64_t n, void *stream);
int launch_degrid(const InterpArgs &a, void *stream);
int launch_grid(const InterpArgs &a, void *stream);
int launch_data_dual(const DualArgs &a, void *stream);

}  // namespace data
}  // namespace fhs

struct fhs_data_plan {
  int ny = 0, nx = 0, L = 0, K1 = 0, K2 = 0;
  int64_t m = 0;                       // visibilities over all channels
  std::vector<int64_t> voff;           // [L + 1]
  // host tables, copied into the workspace when it is attached
  std::vector<fhs::data::VisInfo> info;
  std::vector<float> w;                // [m][2 J]
  std::vector<float> s1, s2;           // Z scaling per axis
  std::vector<fhs::data::float2v> tw1, tw2;  // exp(-2 pi i k / K), k < K / 2, per axis
  std::vector<double> density_inv;     // inverse sampling density per visibility
  std::vector<int32_t> perm;           // visibilities sorted by (channel, grid tile)
  std::vector<fhs::data::GridItem> items;
  int wexp = 0;                        // every product of two interpolation weights is below 2^wexp
  // workspace layout (bytes)
  int64_t off_a = 0, off_b = 0, off_v1 = 0, off_v2 = 0, off_p = 0, off_info = 0, off_w = 0, off_s1 = 0,
          off_s2 = 0, off_tw1 = 0, off_tw2 = 0, off_voff = 0, off_perm = 0, off_items = 0, off_part = 0,
          off_chs = 0, ws_bytes = 0;
  void *ws = nullptr;
};
