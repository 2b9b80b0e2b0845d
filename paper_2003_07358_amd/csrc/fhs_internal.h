// Internal declarations of libfhs: plan layout and kernel argument blocks.
// Not part of the ABI (see include/fhs.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fhs.h"

namespace fhs {

constexpr int kBases = 8;          // db1 .. db8 (the Dirac basis is handled apart)
constexpr int kMaxTap = 16;        // db8 has 16 taps
constexpr int kMaxLevels = 6;
constexpr int kMaxFacetAxis = 64;  // facets per axis
constexpr int kMaxLc = 64;         // channels per sub-cube
#ifndef FHS_ANA_THREADS
#define FHS_ANA_THREADS 512        // analysis workgroup size bound (256 or 512)
#endif
constexpr int kDiracThreads = 256;  // workgroup size of the Dirac-band kernel
constexpr int kDiracE = 8;          // pixels per thread in flight there
constexpr int kAnaLaneSeg = 512;   // LDS words of one staged W row run (TKX L <= threads per workgroup)
constexpr int kAnaThSeg = 128;     // LDS words of one staged theta segment (C TKX <= threads / 4)
static_assert(FHS_ANA_THREADS <= kAnaLaneSeg, "analysis W segments hold up to one word per thread");
#ifndef FHS_SYN_THREADS
#define FHS_SYN_THREADS 512        // synthesis workgroup size bound (256 or 512)
#endif

// ---------------------------------------------------------------- error state
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// ---------------------------------------------------------------- host math
// Daubechies scaling filter dbN (2N taps, long double), spectral factorisation.
std::vector<long double> daubechies(int N);
void chi_mean_std(double k, double *m, double *s);

// ---------------------------------------------------------------- kernel args
// One wavelet basis at one level of the analysis.
struct AnaBand {
  const float *in;     // input band [in_ny][in_nx][L]
  float *ll_out;       // low-low output [Ky][Kx][L] (workspace) or null on the last level
  int in_ny, in_nx;
  int in_natural;      // 1: input is the cube (natural channel order), 0: positions
  int Ky, Kx;
  int strips, yblocks;
  int ntap;
  int64_t off[4];      // first coefficient row of lh, hl, hh, ll (ll: last level, else -1)
  int ky_begin, ky_end, kx_begin, kx_end;  // coefficients computed (the whole band unless per facet);
                                            // for the Dirac band: the pixel rectangle
  int32_t own_r, own_c;  // offsets in AnaArgs::own of the owner facet row of each coefficient row / column
};

struct AnaArgs {
  AnaBand b[kBases + 1];      // [8] = Dirac (elementwise; strips = its workgroups)
  float *w;
  float *theta;               // read (mode 1) or written (mode 2)
  const double *mu;           // [C] thresholds mu_c (mode 1) or upsilon_c (mode 2)
  double inv_kappa;
  int64_t I;
  int64_t theta_bytes;        // C * I * 4 (< 2^31)
  int L, C, Lc, Lcp, tkx1, tky;
  int mode;                   // 0: write Psi^dagger x; 1: l21 dual update; 2: l21 weights;
                              // 3: l21 dual update of the rows owned by selected facets only
  int P;                      // steps per LDS phase
  int lds_row;                // words per staged input row ([sub-cube][column][lane slot], 16-tap width)
  int lds_wv, lds_th;         // offsets (words) of the W and theta areas in a phase buffer
  int lds_buf;                // words per phase buffer
  int lds_tab;                // offset (words) of the row copy table (after both buffers)
  int lds_words;              // LDS words of the launch
  int vec4;                   // 1: channel counts allow 16-byte copies (L and Lc multiples of 4)
  int direct;                 // 1: taps, W and theta loaded straight into registers (no LDS staging)
  int tiles_per_xcd;          // tiles walked by each XCD
  int nbase_wg;               // 64 * tiles_per_xcd workgroups for the wavelet bases
  int tile_major;             // launch order: 1 the 8 bases of a tile back to back, 0 basis-major
  int f32;                    // 1: FP32 accumulation of the filters (mixed-precision form, mode 1)
  const int32_t *active;      // [C] sub-cubes whose W (mode 1) or theta (mode 2) may change; null: all
  const uint8_t *sel;         // mode 3: [C][Q] facets whose owned rows are updated
  const uint8_t *own;         // mode 3: owner facet row / column tables (plan workspace)
  int qy, qx;                 // facets per axis
};

// One wavelet basis at one level of the synthesis (levels >= 2): writes the
// low-low band of the level above into the workspace.
struct SynBand {
  const float *ll;            // [Ky][Kx][L]
  const float *lh, *hl, *hh;  // [Ky][Kx][L]
  float *out;                 // [ny][nx][L]
  int Ky, Kx, ny, nx;
  int strips, yblocks;
  int ntap;
  int y_begin, y_end, x_begin, x_end;  // output samples computed (all unless per facet)
};

struct SynArgs {
  SynBand b[kBases];
  int wg_prefix[kBases + 1];
  int L, Lcp, C, Lc, tk, ty;  // tk: coefficient columns per workgroup (2 tk outputs)
};

// Level 1 of the synthesis for all bases at once, plus the Dirac basis,
// accumulated into the image: x = beta x + alpha / 3 (sum_b ... + w_dirac).
struct SynFinalArgs {
  SynBand b[kBases];          // out, strips, yblocks unused per basis
  float *dirac;               // [ny][nx][L] (positions); updated in place when fused
  float *x;                   // [ny][nx][L] natural channel order
  // fused Dirac-band dual update (first group): W_d <- shrink(W_d + xin / 3)
  // before W_d enters the output; null xin: W_d is read as it is
  const float *xin;           // [ny][nx][L] natural channel order
  const float *theta;         // [C][I] weights (the Dirac rows at dirac_row)
  const double *mu;           // [C]
  double inv_kappa;
  int64_t I, dirac_row;       // coefficient rows per sub-cube; first row of the Dirac band
  int64_t theta_bytes;        // C * I * 4 (< 2^31)
  const int32_t *active;      // [C] sub-cubes whose Dirac rows the fused update may change; null: all
  float alpha, beta;
  int contig;                 // 1: sub-cube c holds the contiguous channels [c Lc, (c + 1) Lc)
  int ny, nx, L, Lcp, C, Lc, tk, ty, strips, yblocks;
  int y_begin, y_end, x_begin, x_end;  // output pixels computed (all unless per facet)
};

// Facet geometry for the nuclear kernels (Sec. 2.4.2).
struct NucGeom {
  int ny, nx, L, C, Lc, qy, qx, oy, ox;  // Lc: columns of a facet matrix
  // spectral layout: spec 0 = interleaved sub-cubes (column ch of sub-cube c
  // is channel c + ch C); spec 1 = contiguous blocks of sb channels whose
  // facet columns start so channels before the block (channel c sb - so + ch,
  // weighted by the spectral ramp)
  int spec, sb, so;
  int ty[kMaxFacetAxis + 1], tx[kMaxFacetAxis + 1];  // tile bounds
  int py[kMaxFacetAxis + 1], px[kMaxFacetAxis + 1];  // prefix sums of window heights / widths
  int64_t p_sub;  // floats of P per sub-cube
};

struct NucArgs {
  NucGeom g;
  const float *x;            // cube [ny][nx][L]
  float *p;                  // packed P
  double *gram;              // [facets][chunks][Lc16][Lc16] partial Gram matrices
  double *kmat;              // [facets][Lc16][Lc16] K = V Diag(h) V^T
  double *sig;               // [facets][Lc] singular values (descending)
  const double *theta_bar;   // [facets][Lc]
  const double *mu_bar;      // [facets] (or upsilon_bar for the weights)
  double *theta_bar_out;     // reweighting output or null
  double inv_zeta;
  int chunks;                // window-row chunks per facet (grid.x of the Gram / reconstruction kernels)
  int chunk_wrows;           // window rows per chunk
  int seg;                   // pixels per staged segment
  int lc16;                  // Lc rounded up to 16
  int mode;                  // 0: dual update; 1: weights only
  int bf16;                  // 1: Gram of BF16-rounded Z on BF16 MFMA, FP32 accumulation (mixed form)
  int q0;                    // first spatial facet of the launch (blockIdx.y offset)
  int eig_q;                 // -1: eig over all C*Q facets; else facets c*Q + eig_q, c < C
  const int32_t *active;     // [C] sub-cubes whose P (mode 0) or theta_bar (mode 1) may change; null: all
  const uint8_t *sel;        // [C][Q] facets whose P is updated (mode 0), or null: all
  unsigned *diag;            // [2] counters: eigendecompositions not converged, non-finite Grams (or null)
};

struct GatherArgs {
  NucGeom g;
  const float *p;
  float *grad;
  double zeta;
  float beta;
  int y_begin, y_end, x_begin, x_end;  // pixels updated (the image unless per facet)
};

// Data-fidelity dual (identity operator), primal update and relative variation.
struct ClosureArgs {
  float *x, *xcheck, *v;
  const float *y, *grad;
  const double *eps;   // [L] l2-ball radii
  double *part;        // [nblocks][2 L] block partial sums per channel (workspace)
  double *factor;      // [L] dual scale factors (workspace)
  double *xi;          // [C] relative variation of each sub-cube in this iteration
  const int32_t *active;  // [C] sub-cubes whose x, xcheck, v may change; null: all
  double tau;
  int64_t npix, ppb;   // pixels, pixels per block
  int L, C, nblocks;
  int contig;          // 1: sub-cube c holds the contiguous channels [c L / C, (c + 1) L / C)
};

struct SnrArgs {
  const float *ref, *x;  // [N][L] reference and estimate
  const double *eps;     // [L] noise levels for the log-scale metric, or null
  double *part;          // [nblocks][4][L] block partial sums (workspace)
  double *snr, *snr_log; // [L] outputs, or null (snr_log written only with eps)
  double *sums;          // [2][L] raw sums of r^2 and (r - x)^2 per channel, or null
  int64_t npix, ppb;
  int L, nblocks;
};

// ---------------------------------------------------------------- launchers
int launch_analysis(const AnaArgs &a, int nthreads, bool first, void *stream);
int launch_analysis_m0(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream);
int launch_analysis_m1(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream);
int launch_analysis_m1f(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream);
int launch_analysis_m2(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream);
int launch_analysis_m3(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream);
int launch_synthesis(const SynArgs &a, int nthreads, void *stream);
int launch_synthesis_final(const SynFinalArgs &a, int nthreads, int group, void *stream);
int launch_nuc_gram(const NucArgs &a, int nspatial, void *stream);
int launch_nuc_eig(const NucArgs &a, int nfacets, void *stream);
int launch_nuc_recon(const NucArgs &a, int nspatial, void *stream);
int launch_nuc_gather(const GatherArgs &a, void *stream);
int launch_closure(const ClosureArgs &a, void *stream);
int launch_snr(const SnrArgs &a, void *stream);

// Compute sequences shared by the entry points.  `active` ([C] int32 device
// flags, or null for all) restricts every state write to the sub-cubes whose
// flag is set: the other sub-cubes keep their P, W, theta, theta_bar (and, in
// the closure, x, xcheck, v) bit for bit.
int facet_prox_step(const fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                    const double *theta_bar, const double *mu, const double *mu_bar, double zeta, double kappa,
                    float *grad, void *stream, const int32_t *active, const uint8_t *sel = nullptr);
int reweight(const fhs_plan *p, const float *x, const double *upsilon, const double *upsilon_bar, float *theta,
             double *theta_bar, void *stream, const int32_t *active);
// Workspace base of the compute sequences: the plan's, or the static scratch
// while fhs_facet_prox_step_noalloc runs on this thread.
void *ws_base(const fhs_plan *p);

}  // namespace fhs

// ---------------------------------------------------------------- the plan
struct fhs_plan {
  fhs_config cfg{};
  int L = 0, C = 1, Lc = 0, Q = 0, Lcp = 0, lc16 = 0;
  int so = 0, Ln = 0;                      // spectral overlap; columns of a facet matrix (Lc + so)
  std::vector<int> ty, tx;                 // tile bounds
  struct Facet {
    int c, sy, sx, ty0, ty1, tx0, tx1, wy0, wy1, wx0, wx1;
    int64_t poff, rows;
  };
  std::vector<Facet> facets;
  int64_t n_p = 0, p_sub = 0;
  struct Band { int64_t rows, cols, off; int level; };
  std::vector<Band> bands;
  int64_t I = 0;
  // per basis b, level j (0-based): input dims and band dims
  int in_ny[fhs::kBases][fhs::kMaxLevels], in_nx[fhs::kBases][fhs::kMaxLevels];
  int Ky[fhs::kBases][fhs::kMaxLevels], Kx[fhs::kBases][fhs::kMaxLevels];
  int64_t band_first[fhs::kBases];         // index into `bands` of the basis' first band
  // per basis and level, the Q_axis + 1 boundaries of the coefficients each
  // facet owns (used by the per-facet execution form)
  std::vector<int> own_y[fhs::kBases][fhs::kMaxLevels], own_x[fhs::kBases][fhs::kMaxLevels];
  // the same as tables (uint8 owner facet row of every coefficient row, owner
  // facet column of every coefficient column; the Dirac band: the tiles),
  // copied into the workspace at ws_own when it is attached
  std::vector<uint8_t> own_tab;
  int32_t own_r[fhs::kBases][fhs::kMaxLevels], own_c[fhs::kBases][fhs::kMaxLevels];
  int32_t own_dr = 0, own_dc = 0;
  float h[fhs::kBases][fhs::kMaxTap], g[fhs::kBases][fhs::kMaxTap];
  int ntap[fhs::kBases];
  // workspace layout (bytes)
  int64_t ws_ll[fhs::kBases][fhs::kMaxLevels];
  int64_t ws_gram = 0, ws_kmat = 0, ws_sig = 0, ws_red = 0, ws_factor = 0, ws_ctl = 0, ws_active = 0, ws_diag = 0,
          ws_own = 0;
  int64_t ws_bytes = 0;
  int64_t red_ppb = 0;                     // closure: pixels per block
  int red_blocks = 0;                      // closure: blocks
  int gram_chunks = 0, max_rows = 0;       // Gram partial slots per facet (workspace capacity)
  int max_hy = 0, max_hx = 0;               // largest window
  int nuc_chunk_min = 1;                    // smallest window-row chunk the workspace allows
  fhs_tuning tune{};                        // launch shapes
  void *ws = nullptr;
  int64_t ws_given = 0;
  // second stream and fork / join events: the nuclear chain runs beside the
  // wavelet chain (created when the workspace is attached; null = one stream)
  void *side = nullptr, *ev_fork = nullptr, *ev_join = nullptr;
  // optional per-kernel event timing (diagnostics)
  mutable int prof_kernel = -1;
  mutable std::vector<void *> prof_events;  // hipEvent_t pairs
  mutable int prof_next = 0;
};

namespace fhs {
// LDS bytes of one nuclear reconstruction workgroup for segments of S pixels.
int64_t nuc_recon_lds(const fhs_plan *p, int S);
// Records the start / stop events around one launch when profiling `kid`.
void prof_begin(const fhs_plan *p, int kid, void *stream);
void prof_end(const fhs_plan *p, int kid, void *stream);
void prof_release(fhs_plan *p);
}  // namespace fhs
