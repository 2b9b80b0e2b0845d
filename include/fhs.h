/*
 * fhs.h -- C ABI of the facet-wise regularization step of Faceted HyperSARA
 * (Thouvenin, Abdulaziz, Dabbech, Repetti, Wiaux, arXiv:2003.07358) on
 * AMD Instinct MI355X (gfx950).
 *
 * Scope.  One PDFB iteration of Algorithm 2 updates, for every spectral
 * sub-cube c and spatial facet q, two dual variables and aggregates their
 * contributions into the primal gradient:
 *
 *   nuclear  (Alg. 2, nuclear-norm dual update; Table 1 SVT):
 *     P_{c,q} <- (I - prox_{zeta^-1 mu_bar_{c,q} ||.||_{*,theta_bar_{c,q}}})(P_{c,q} + D_q S~_q Xcheck_c)
 *   l21      (Alg. 2, l21 dual update; Table 1 row shrink):
 *     W_{c,q} <- (I - prox_{kappa^-1 mu_c ||.||_{2,1,theta_{c,q}}})(W_{c,q} + Psi_q^dagger S_q Xcheck_c)
 *   gather   (Alg. 2, aggregation, facet part):
 *     G_c = sum_q zeta S~_q^T D_q P_{c,q} + kappa S_q^T Psi_q W_{c,q}
 *
 * Psi^dagger is the SARA dictionary (Sec. 2.3.1): Daubechies db1..db8 at
 * `levels` levels plus the Dirac basis, divided by 3.  The faceted transform is
 * exactly the global one (Sec. 2.4.2), so W is held in the global coefficient
 * layout and every facet owns a rectangle of each band.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays.   Every array argument of a compute call is a DEVICE pointer owned by
 *           the caller (e.g. a torch tensor).  The library never frees, never
 *           allocates device memory in a compute call and never synchronises
 *           the host; every compute call is asynchronous on `stream`
 *           (a hipStream_t passed as void*, NULL = the null stream).
 * Cube.     X, Xcheck, G: float32 [ny][nx][L], channels contiguous (pixels are
 *           rows and channels columns of the N x L matrix of Sec. 2.2).
 * Sub-cubes. Channel-interleaved (Sec. 2.4.1): sub-cube c holds the channels
 *           c, c + C, c + 2C, ...; C must divide L, L_c = L / C <= 64.
 *           Channel "position" p = c * L_c + l stands for channel c + l * C.
 * P.        float32, packed per facet f = c * Q + q in that order, each facet a
 *           row-major [ny~_q][nx~_q][L_c] block (offsets from fhs_plan_facet).
 * W.        float32 [I][L]: coefficient row i (a position in a band), then the
 *           L channel positions p (sub-cube-major).  Band order: db1 .. db8,
 *           each as (lh, hl, hh) for level 1 .. levels, then ll of the last
 *           level; finally the Dirac band [ny][nx].  I = fhs_sizes.n_coef.
 * theta.    float32 [C][I]: one l21 weight per coefficient row and sub-cube.
 * theta_bar float64 [C*Q][L_c]: nuclear weights of facet f, paired with the
 *           singular values in descending order.
 * mu        float64 [C]      (mu_c of eq. heuristic_fhs_sparsity).
 * mu_bar    float64 [C*Q]    (mu_bar_{c,q} of eq. heuristic_fhs_low_rank).
 * Workspace. Caller-owned device memory of fhs_sizes.workspace_bytes bytes,
 *           attached once with fhs_plan_set_workspace; compute calls use it as
 *           scratch, so calls that share a plan must not overlap in time.
 * Errors.   Every int-returning function returns FHS_OK (0) or a negative
 *           code; fhs_last_error() returns a thread-local message.  No C++
 *           exception crosses the ABI.  A HIP launch error is reported as
 *           FHS_EHIP; execution errors surface on the stream, as usual.
 */
#ifndef FHS_H
#define FHS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FHS_OK 0
#define FHS_EINVAL (-1)         /* bad argument (null pointer, size, range) */
#define FHS_EHIP (-2)           /* a HIP runtime call failed */
#define FHS_ENOMEM (-3)         /* host allocation failed */
#define FHS_EUNSUPPORTED (-4)   /* valid but unsupported configuration */
#define FHS_ENOWORKSPACE (-5)   /* compute call before fhs_plan_set_workspace */

typedef struct fhs_plan fhs_plan;   /* opaque; immutable geometry after creation */

/* Precision forms (fhs_config.precision). */
#define FHS_PRECISION_FP32 0   /* FP32 storage; wavelet filters, Gram and reconstruction
                                  accumulated in FP64 (every output within 1e-5 of FP64)  */
#define FHS_PRECISION_MIXED 1  /* the l21 update's wavelet filters accumulated in FP32; the
                                  facet Gram of BF16-rounded Z on BF16 MFMA with FP32
                                  accumulation; eigendecomposition, sigma scaling and the
                                  reconstruction in FP64 as above.  The weights
                                  (fhs_reweight) and the synthesis are not affected.  Error
                                  (vs FP64): W+ about 1e-5, P+ growing as 2^-8 kappa^2 with
                                  kappa = sigma_1 / min_j t_j of the facet               */

typedef struct {
  int32_t ny, nx;        /* image size, N = ny * nx                                  */
  int32_t nchan;         /* L, channels of the cube                                  */
  int32_t qy, qx;        /* spatial facet grid, Q = qy * qx (Sec. 2.4.2)            */
  int32_t n_sub;         /* C, interleaved spectral sub-cubes (Sec. 2.4.1); 1 = none */
  int32_t overlap_y;     /* low-rankness overlap in pixels toward the top (Sec. 2.4.2) */
  int32_t overlap_x;     /* ... toward the left                                      */
  int32_t levels;        /* wavelet decomposition levels (1..6; 4 in the paper)      */
  int32_t precision;     /* FHS_PRECISION_FP32 (0) or FHS_PRECISION_MIXED (1)         */
  int32_t spectral_overlap; /* o: 0 = the paper's interleaved, independent sub-cubes.
                            o > 0 (a reading beyond the paper, FP32 form, C >= 2,
                            o <= L/C): C contiguous blocks of L/C channels (the l21
                            rows), each low-rankness facet also taking the o channels
                            before its block, with the spatial window's triangular
                            ramp applied along channels (Sec. 2.4.2 rule on the
                            spectral axis), so the blocks' weights sum to one per
                            channel.  A facet's P then has L/C + o columns, the
                            window's channels in order; for the first block the
                            first o columns lie before channel 0 and are structural
                            zeros (pass zeros; they stay zero).  theta_bar likewise
                            has L/C + o weights per facet (for the first block the
                            first L/C apply).  The sub-cubes are no longer
                            independent: the PDFB closure and solve reject it.     */
} fhs_config;

typedef struct {
  int64_t n_x;              /* floats of X, Xcheck, G: ny*nx*L                 */
  int64_t n_p;              /* floats of the packed P                          */
  int64_t n_coef;           /* I, coefficient rows of Psi^dagger               */
  int64_t n_w;              /* floats of W: I * L                              */
  int64_t n_theta;          /* floats of theta: C * I                          */
  int64_t n_facets;         /* C * Q                                           */
  int64_t n_theta_bar;      /* doubles of theta_bar: C * Q * L_c (+ o, see
                               spectral_overlap)                                */
  int64_t n_bands;          /* bands of Psi^dagger: 8 * (3 levels + 1) + 1     */
  int64_t workspace_bytes;  /* bytes for fhs_plan_set_workspace                */
} fhs_sizes;

/* ---------------------------------------------------------------- host only */

/* Library version (major * 100 + minor). */
int fhs_version(void);

/* Thread-local message of the last failing call ("" if none). */
const char *fhs_last_error(void);

/* Daubechies extremal-phase scaling filter dbN, N = 1..8 (the eight wavelet
 * bases of the SARA dictionary, Sec. 2.3.1), derived by the library by
 * spectral factorisation of the Daubechies polynomial.  Writes 2N doubles to
 * the HOST array h_out.  High-pass: g[m] = (-1)^m h[2N-1-m]. */
int fhs_filter(int32_t N, double *h_out);

/* Mean and standard deviation of a chi distribution with k degrees of
 * freedom (used by eqs. heuristic_hypersara_sparsity and heuristic_fhs_sparsity).
 * HOST pointers. */
int fhs_chi_mean_std(double k, double *mean, double *std_dev);

/* Builds the geometry: tiles t_s = floor(s n / Q); low-rankness facets
 * extended by the overlap toward top/left, edge facets keeping the tile size
 * (Sec. 2.4.2); band sizes of the zero-extended expansive transform; packed
 * offsets; workspace size.  Host memory only.  *out receives the plan. */
int fhs_plan_create(const fhs_config *cfg, fhs_plan **out);
void fhs_plan_destroy(fhs_plan *plan);
int fhs_plan_sizes(const fhs_plan *plan, fhs_sizes *out);

/* Facet f (0 <= f < C*Q) as 12 int64 on the HOST:
 * {c, sy, sx, tile_y0, tile_y1, tile_x0, tile_x1,
 *  win_y0, win_y1, win_x0, win_x1, p_offset (floats into the packed P)}. */
int fhs_plan_facet(const fhs_plan *plan, int32_t f, int64_t out[12]);

/* Band k (storage order) as 4 int64 on the HOST: {rows, cols, first
 * coefficient row, level (0 for the Dirac band)}. */
int fhs_plan_band(const fhs_plan *plan, int32_t k, int64_t out[4]);

/* Regularisation parameters from the noise level sigma_bar_c (HOST arrays):
 * mu_c = sigma_bar_c (m_chi(L_c) + s_chi(L_c))            (eq. heuristic_fhs_sparsity)
 * mu_bar_{c,q} = sigma_bar_c sqrt(N~_q L_c / min(N~_q, L_c)) (eq. heuristic_fhs_low_rank)
 * sigma_bar [C] in, mu [C] out, mu_bar [C*Q] out. */
int fhs_plan_heuristics(const fhs_plan *plan, const double *sigma_bar, double *mu, double *mu_bar);

/* Launch shapes of the kernels.  They change speed, not the computation: the
 * wavelet outputs are bitwise the same for every valid setting; the nuclear
 * Gram sums follow the row chunking, so P and G may differ in the last bits.
 * For a fixed setting every call is bitwise reproducible. */
typedef struct {
  int32_t ana_rows[6];     /* coefficient rows per analysis workgroup, per level (8..256) */
  int32_t ana_phase;       /* upper bound on steps per LDS phase of the analysis (1, 2, 4) */
  int32_t syn_rows;        /* output rows per synthesis workgroup, levels >= 2 (16..256) */
  int32_t fin_rows;        /* output rows per level-1 synthesis workgroup (16..512) */
  int32_t nuc_seg;         /* pixels per staged segment of the nuclear kernels (16, 32, 64) */
  int32_t nuc_chunk_rows;  /* window rows per nuclear workgroup (>= the plan's minimum) */
  int32_t concurrent;      /* 1: the nuclear chain runs on a second stream beside the wavelet chain */
  int32_t ana_direct;      /* bit j set: the analysis of level j+1 loads taps, W and theta straight
                              into registers (no LDS); bit mask over the levels */
  int32_t fin_waves;       /* wavefronts per level-1 synthesis workgroup (4, 6 or 8) */
  int32_t ana_order;       /* bit j set: the analysis of level j+1 launches the 8 bases of a tile
                              back to back (tile-major), else basis-major; bit mask over the levels */
} fhs_tuning;

/* Current launch shapes (defaults after fhs_plan_create). HOST pointer. */
int fhs_plan_get_tuning(const fhs_plan *plan, fhs_tuning *out);
/* Replaces the launch shapes; FHS_EINVAL (plan unchanged) if a field is out
 * of range.  Not to be called while compute calls of the plan are in flight. */
int fhs_plan_set_tuning(fhs_plan *plan, const fhs_tuning *tuning);

/* Autotuner: times fhs_facet_prox_step for candidate launch shapes, one field
 * at a time (coordinate descent, `reps` steps per candidate, HIP events on
 * `stream`), keeps the fastest and returns with the plan set to it.  The
 * arguments are those of fhs_facet_prox_step; p_inout, w_inout and grad are
 * overwritten with unspecified values (pass scratch copies).  Synchronises
 * the host with `stream`; a setup call, not a compute call. */
int fhs_plan_autotune(fhs_plan *plan, const float *xcheck, float *p_inout, float *w_inout,
                      const float *theta, const double *theta_bar, const double *mu,
                      const double *mu_bar, float *grad, int32_t reps, void *stream);

/* Attaches caller-owned device scratch of at least fhs_sizes.workspace_bytes
 * bytes (256-byte aligned).  The plan keeps the pointer, not the memory. */
int fhs_plan_set_workspace(fhs_plan *plan, void *dev_ptr, int64_t bytes);

/* ---------------------------------------------------------------- compute */

/* w = Psi^dagger x (Sec. 2.3.1): all nine bases, divided by 3; x [ny][nx][L]
 * in natural channel order, w [I][L] in channel positions. */
int fhs_sara_analysis(const fhs_plan *plan, const float *x, float *w, void *stream);

/* x = beta x + alpha Psi w, Psi the adjoint of Psi^dagger (Alg. 2, facet synthesis
 * summed over facets). */
int fhs_sara_synthesis(const fhs_plan *plan, const float *w, float *x, float alpha, float beta,
                       void *stream);

/* l21 dual update of every facet (Alg. 2, l21 dual update) and its
 * gather: for every coefficient row i and sub-cube c,
 *   u = W_i + [Psi^dagger Xcheck_c]_i,  W_i <- u min(1, (mu_c / kappa) theta_{c,i} / ||u||_2)
 *   (W_i <- 0 when u = 0),
 * then grad = beta grad + kappa Psi W.  W is updated in place; grad must not
 * alias xcheck or w_inout. */
int fhs_l21_dual_update(const fhs_plan *plan, const float *xcheck, float *w_inout,
                        const float *theta, const double *mu, double kappa, float *grad,
                        float beta, void *stream);

/* Weighted nuclear-norm dual update of every facet (Alg. 2) and its gather:
 * Z = P_f + D_q S~_q Xcheck_c (N~_q x L_c),
 * thresholds t_j = (mu_bar_f / zeta) theta_bar_{f,j} paired with the singular
 * values s_1 >= s_2 >= ..., and
 *   P_f <- Z - prox(Z) = U Diag(min(s_j, t_j)) V^T = Z V Diag(min(1, t_j / s_j)) V^T,
 * then grad = beta grad + zeta sum_f S~_q^T D_q P_f (facet
 * back-projection and aggregation).  P is updated in place. */
int fhs_nuclear_dual_update(const fhs_plan *plan, const float *xcheck, float *p_inout,
                            const double *theta_bar, const double *mu_bar, double zeta,
                            float *grad, float beta, void *stream);

/* Both dual updates and the full facet part of the aggregation (Alg. 2,
 * facet loop and aggregation):
 *   grad = zeta sum_f S~_q^T D_q P_f + kappa Psi W   (grad overwritten). */
int fhs_facet_prox_step(const fhs_plan *plan, const float *xcheck, float *p_inout,
                        float *w_inout, const float *theta, const double *theta_bar,
                        const double *mu, const double *mu_bar, double zeta, double kappa,
                        float *grad, void *stream);

/* Randomized form of the step (Sec. 3.2: a random subset of the facet dual
 * variables is updated at an iteration).  select: device uint8 [C][Q]
 * (facet descriptor order f = c Q + q), drawn by the caller; nonzero updates
 * the duals of facet f: P_f, and the l21 rows facet q owns in sub-cube c in
 * every band (its coefficients of the faceted transform, Sec. 2.4.2; the
 * Dirac rows of its tile).  The other facets keep their P and W bit for bit.
 * grad is then the aggregation of every facet's current duals, as in
 * fhs_facet_prox_step (overwritten).  Other arguments as there; every
 * selected facet gets the same result as fhs_facet_prox_step gives it. */
int fhs_facet_prox_step_select(const fhs_plan *plan, const float *xcheck, float *p_inout,
                               float *w_inout, const float *theta, const double *theta_bar,
                               const double *mu, const double *mu_bar, double zeta, double kappa,
                               const uint8_t *select, float *grad, void *stream);

/* The same step in the per-facet execution form (the paper's organisation:
 * one facet at a time, Sec. 2.4 and Fig. 4): every operator is launched once
 * per spatial facet on the coefficients / pixels / window rows that facet
 * owns, in raster order (analysis level by level, synthesis coarse to fine,
 * the nuclear update facet by facet, then the gather tile by tile), on
 * `stream` only.  Same arguments and the same results as fhs_facet_prox_step
 * (bitwise for the wavelet part); kept as the baseline the batched form is
 * measured against. */
int fhs_facet_prox_step_plain(const fhs_plan *plan, const float *xcheck, float *p_inout,
                              float *w_inout, const float *theta, const double *theta_bar,
                              const double *mu, const double *mu_bar, double zeta, double kappa,
                              float *grad, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * step as fhs_facet_prox_step, same arguments and results (bit for bit), but
 * its scratch is the library's own static device array of
 * fhs_noalloc_scratch_bytes() bytes (32 MiB; each GPU the library runs on
 * holds one until the process ends) instead of an attached workspace, so no
 * workspace needs to be attached and nothing is allocated, by this call or
 * before it.  Returns FHS_EUNSUPPORTED, without launching anything, when the
 * plan's workspace (fhs_sizes.workspace_bytes) exceeds the scratch.  Every
 * call on one GPU shares that GPU's scratch: calls that overlap in time on
 * one GPU race (serialise them, e.g. on one stream).  The scratch keeps the
 * previous call's contents; the step writes every scratch word before it
 * reads it, so nothing needs clearing. */
int fhs_facet_prox_step_noalloc(const fhs_plan *plan, const float *xcheck, float *p_inout,
                                float *w_inout, const float *theta, const double *theta_bar,
                                const double *mu, const double *mu_bar, double zeta, double kappa,
                                float *grad, void *stream);
/* Bytes of the static scratch of fhs_facet_prox_step_noalloc (host call). */
int64_t fhs_noalloc_scratch_bytes(void);

/* Reweighting weights from the previous iterate X^(t) (Alg. 1,
 * weight updates):
 *   theta_bar_{f,j} = upsilon_bar_f / (s_j(D_q S~_q X_c) + upsilon_bar_f)  (eq. facet_hypersara_rank)
 *   theta_{c,i}     = upsilon_c / (||[Psi^dagger X_c]_i||_2 + upsilon_c)    (eq. facet_hypersara_sparsity)
 * upsilon [C] and upsilon_bar [C*Q] are float64 device arrays. */
int fhs_reweight(const fhs_plan *plan, const float *x, const double *upsilon,
                 const double *upsilon_bar, float *theta, double *theta_bar, void *stream);

/* ---------------------------------------------------------------- PDFB iteration */

/* The rest of an iteration of Algorithm 2 around the facet step, with the
 * identity as measurement operator (a denoising stand-in for the
 * data-fidelity block, whose operator is outside this library), U = I and
 * eta = 1:
 *   v      <- (I - proj_{B(y_l, eps_l)})(v + xcheck)   per channel l (Table 1)
 *   x+      = max(0, x - tau (grad + v))               (primal update, Table 1)
 *   xcheck <- 2 x+ - x,   x <- x+                      (extrapolation)
 *   xi[c]   = ||x+_c - x_c||_F / ||x_c||_F             (relative variation of
 *             spectral sub-cube c, channels c, c + C, ...; +inf if x_c = 0;
 *             Alg. 2 solves each sub-problem on its own)
 * x, xcheck, v, y, grad: float32 [ny][nx][L] (natural channel order); eps:
 * float64 [L]; xi: float64 [C].  All device pointers; x, xcheck, v are
 * updated in place and must not alias y or grad.  The channel norms and xi
 * are accumulated in float64 in a fixed order (bitwise reproducible).  Uses
 * the plan's workspace. */
int fhs_pdfb_closure(const fhs_plan *plan, float *x, float *xcheck, float *v, const float *y,
                     const double *eps, const float *grad, double tau, double *xi, void *stream);

/* Reconstruction quality (Sec. 4.3), per channel l of the plan's cube:
 *   snr[l]     = 20 log10(||x_ref_l||_2 / ||x_ref_l - x_l||_2)
 *   snr_log[l] = the same on log10(z / eps_l + 1) of both images (term-wise)
 * in dB, +inf where the estimate equals the reference.  x_ref, x: float32
 * [ny][nx][L] (natural channel order), device; eps: float64 [L] device noise
 * levels, or NULL to skip the log-scale metric (then snr_log may be NULL);
 * snr, snr_log: float64 [L] device outputs.  Sums in float64, fixed order
 * (bitwise reproducible).  Images must be non-negative where the log-scale
 * metric is taken (otherwise it is NaN).  Uses the plan's workspace. */
int fhs_snr(const fhs_plan *plan, const float *x_ref, const float *x, const double *eps, double *snr,
            double *snr_log, void *stream);

/* Everything one PDFB iteration touches (device pointers, caller-owned). */
typedef struct {
  float *x;                 /* X [ny][nx][L]                                    */
  float *xcheck;            /* Xcheck [ny][nx][L]                               */
  float *p;                 /* nuclear duals, packed (see P above)              */
  float *w;                 /* l21 duals [I][L]                                 */
  float *v;                 /* data-fidelity dual [ny][nx][L]                   */
  const float *y;           /* data [ny][nx][L]                                 */
  const double *eps;        /* l2-ball radius per channel [L]                   */
  const float *theta;       /* [C][I]                                           */
  const double *theta_bar;  /* [C*Q][L_c]                                       */
  const double *mu;         /* [C]                                              */
  const double *mu_bar;     /* [C*Q]                                            */
  float *grad;              /* facet gradient, overwritten [ny][nx][L]          */
  double *xi;               /* relative variations, C float64 per iteration     */
  double zeta, kappa, tau;  /* dual and primal step sizes (tau > 0)            */
} fhs_pdfb_state;

/* One iteration: fhs_facet_prox_step on xcheck (into grad), then
 * fhs_pdfb_closure, writing xi[iter * C .. iter * C + C - 1]. */
int fhs_pdfb_iteration(const fhs_plan *plan, const fhs_pdfb_state *state, int32_t iter, void *stream);

/* A HIP graph of n_iter consecutive iterations (xi[0 .. n_iter C - 1]), captured
 * on a stream of the library's own and instantiated; it bakes in the
 * pointers of *state and the plan's workspace, so those must outlive it and
 * launches that share them must not overlap.  Fails with FHS_EINVAL while
 * kernel profiling is enabled.  The graph holds no device allocation. */
typedef struct fhs_graph fhs_graph;
int fhs_pdfb_graph_create(const fhs_plan *plan, const fhs_pdfb_state *state, int32_t n_iter,
                          fhs_graph **out);
/* Launches the whole graph on `stream` (asynchronous). */
int fhs_graph_launch(const fhs_graph *graph, void *stream);
void fhs_graph_destroy(fhs_graph *graph);

/* ---------------------------------------------------------------- reweighting solve */

/* Stopping parameters of the outer reweighting loop (Alg. 1) and of each
 * PDFB run inside it (Alg. 2).  The paper's values: max_reweights 5,
 * min_iter 10, max_iter 2000, rw_tol = pdfb_tol = 1e-5, res_factor 1.01. */
typedef struct {
  int32_t max_reweights; /* T: at most this many PDFB runs per sub-cube          */
  double rw_tol;         /* a sub-cube's loop ends once its ||X_c(t+1)-X_c(t)||/||X_c(t)|| <= rw_tol */
  int32_t min_iter;      /* PDFB iterations always performed                    */
  int32_t max_iter;      /* PDFB iteration cap (>= 1 and >= min_iter)           */
  double pdfb_tol;       /* bound on the relative variation xi of the iterate   */
  double res_factor;     /* residual bound ||r|| <= res_factor ||eps||          */
} fhs_solve_params;

typedef struct {
  int32_t runs;          /* reweighting passes made (the most of any sub-cube)  */
  int64_t iterations;    /* PDFB iterations over all sub-cubes and runs         */
} fhs_solve_report;

/* Algorithm 1 with the identity as measurement operator, every array
 * resident on the device.  The spectral sub-cubes are independent
 * sub-problems (Sec. 2.4.1): Alg. 1 loops "for c = 1 to C" around its
 * reweighting loop and Alg. 2 solves one sub-problem, so every sub-cube c has
 * its own pass counter, relative variations and stopping decisions:
 *   t_c = 0, xi_c = +inf
 *   while t_c < max_reweights and xi_c > rw_tol:
 *     theta_c, theta_bar_c <- weights from X_c (as fhs_reweight, with
 *                     upsilon [C] and upsilon_bar [C*Q], float64 device arrays)
 *     X_c(t) <- X_c (kept in x_prev), Xcheck_c <- X_c
 *     PDFB run on sub-cube c while p_c < min_iter, or p_c < max_iter and
 *       (xi_{c,p} > pdfb_tol or ||r_c|| > res_factor ||eps_c||), where
 *       ||r_c||^2 = sum_{l in c} ||y_l - x_l||^2 for the iterate entering the
 *       last iteration (Alg. 2, residual step) and ||eps_c||^2 = sum_{l in c}
 *       eps_l^2
 *     xi_c <- ||X_c - X_c(t)||_F / ||X_c(t)||_F,  t_c <- t_c + 1
 * The sub-cubes still running advance together (one launch per operator
 * covers all of them); a sub-cube that has stopped keeps X, P, W, v, theta
 * and theta_bar bit for bit while the others go on (the kernels read
 * per-sub-cube flags kept in the workspace).  P, W and v are warm-started
 * from one run to the next (they are never reset).  state->theta and
 * state->theta_bar are overwritten (they must be writable device memory),
 * state->xi must hold max_iter * C float64 (iteration p of the current pass
 * writes xi[p C + c]), x_prev is a float32 device array of the cube's size.
 * The loop decides on the host: every iteration ends with a small
 * device-to-host copy (xi and the per-channel residual sums) and a
 * synchronization of `stream`.  Host outputs (each NULL to skip):
 * iters [max_reweights * C] int32, iters[t C + c] = iterations of pass t of
 * sub-cube c (0 if it made no such pass); rw_xi [max_reweights * C] float64,
 * the relative variation that ended each pass (+inf where none); report, the
 * summary.  Uses the plan's workspace. */
int fhs_reweighting_solve(const fhs_plan *plan, const fhs_pdfb_state *state, const double *upsilon,
                          const double *upsilon_bar, float *x_prev, const fhs_solve_params *params,
                          int32_t *iters, double *rw_xi, fhs_solve_report *report, void *stream);

/* ---------------------------------------------------------------- diagnostics */

/* Counters kept in the plan's workspace since it was attached (or last
 * reset): out[0] = nuclear eigendecompositions whose cyclic Jacobi still had
 * off-diagonal energy above 1e-20 of the total after its 40 sweeps (not
 * converged; the step went on with the last rotation), out[1] = facets whose
 * Gram matrix was not finite (NaN or Inf in the input).  HOST out; reads them
 * on `stream` and synchronises it; reset != 0 clears them afterwards.  Not a
 * compute call (do not capture it in a graph). */
int fhs_plan_diagnostics(const fhs_plan *plan, int64_t out[2], int32_t reset, void *stream);

/* Kernel identifiers for fhs_plan_profile. */
#define FHS_K_ANALYSIS_L1 0   /* analysis, level 1 of all bases + Dirac (fused l21 update) */
#define FHS_K_ANALYSIS 1      /* analysis, levels >= 2                                    */
#define FHS_K_SYNTHESIS 2     /* synthesis, levels >= 2                                   */
#define FHS_K_SYNTH_FINAL_A 3 /* synthesis level 1, first group of bases + Dirac          */
#define FHS_K_SYNTH_FINAL_B 4 /* synthesis level 1, second group of bases                 */
#define FHS_K_NUC_GRAM 5
#define FHS_K_NUC_EIG 6
#define FHS_K_NUC_RECON 7
#define FHS_K_NUC_GATHER 8
#define FHS_K_CLOSURE 9       /* data dual + primal update (the four closure kernels)     */
#define FHS_K_COUNT 10

/* Times every launch of kernel `kernel_id` (or none if -1) with HIP events
 * recorded on the launch stream around it.  Creates up to `max_launches`
 * event pairs now (host call; not during compute calls).  Returns FHS_OK. */
int fhs_plan_profile(fhs_plan *plan, int32_t kernel_id, int32_t max_launches);

/* Waits for the recorded events, returns the summed duration (ms) and the
 * number of timed launches since the last read, and resets the counters. */
int fhs_plan_profile_read(fhs_plan *plan, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------- data fidelity
 *
 * The measurement operator of one channel, Phi_l = G_l F Z (Sec. 2.1, eq.
 * model), for a real ny x nx image:
 *   Z  zero-pads the image into a K1 x K2 grid (K = 2 N per axis), pixel n at
 *      grid index (n - N/2) mod K (the image centred on the grid origin),
 *      scaled by 1 / psi^(m / K) per axis (m = n - N/2), psi^ the continuous
 *      Fourier transform of the interpolation kernel;
 *   F  the unnormalised 2D DFT, exp(-2 pi i k.g / K);
 *   G  de-gridding with the 7 x 7 Kaiser-Bessel kernel (Sec. 2.1, Sec. 4.1):
 *      visibility j at the uv-point omega_j (radians per pixel; Phi x then
 *      approximates sum_n x[n] exp(-i omega_j.(n - N/2))) at grid coordinate
 *      t = omega K / (2 pi) sums the 7 x 7 grid points from ceil(t - 7/2),
 *      weights psi(t - k) = I0(beta sqrt(1 - (2 (t - k) / 7)^2)) per axis,
 *      beta = pi sqrt((7/2)^2 (3/2)^2 - 0.8) (Beatty, Nishimura and Pauly).
 * One data block per channel.  FP32 storage and FFT, FP64 interpolation sums
 * and reductions.  Visibilities are complex FP32 (re, im interleaved), all
 * channels concatenated in channel order (channel l from sum_{l' < l} n_vis). */
typedef struct fhs_data_plan fhs_data_plan;  /* opaque */

typedef struct {
  int32_t ny, nx;  /* image size: powers of two, 8 .. 4096                    */
  int32_t nchan;   /* L                                                       */
} fhs_data_config;

/* n_vis: host [L] visibilities per channel; uv: host [sum n_vis][2]
 * (omega_y, omega_x) per visibility, |omega| < 1e6 (the grid wraps).
 * Computes the interpolation tables, the scaling of Z and the inverse
 * sampling density on the host.  FHS_EUNSUPPORTED for non-power-of-two
 * sides or more than 2^31 visibilities. */
int fhs_data_plan_create(const fhs_data_config *cfg, const int64_t *n_vis, const double *uv, fhs_data_plan **out);
void fhs_data_plan_destroy(fhs_data_plan *plan);

/* out[0] = total visibilities, out[1] = workspace bytes, out[2] = K1, out[3] = K2. */
int fhs_data_plan_sizes(const fhs_data_plan *plan, int64_t out[4]);

/* Caller-owned device workspace (256-byte aligned, at least out[1] bytes);
 * the tables are copied into it now (host call, synchronises the device). */
int fhs_data_plan_set_workspace(fhs_data_plan *plan, void *dev_ptr, int64_t bytes);

/* The preconditioner of Sec. 3.2: U_j = 1 / (number of uv-points of channel l
 * in the cell of the oversampled grid nearest to omega_j).  Host [sum n_vis]. */
int fhs_data_preconditioner(const fhs_data_plan *plan, double *u_out);

/* vis = Phi x for every channel.  x: device FP32 [ny][nx][L]; vis: device
 * complex FP32 [sum n_vis]. */
int fhs_nufft_forward(const fhs_data_plan *plan, const float *x, float *vis, void *stream);

/* x = beta x + scale_l Re(Phi_l^dagger v) per channel (scale: device FP64 [L],
 * or null for 1). */
int fhs_nufft_adjoint(const fhs_data_plan *plan, const float *vis, float *x, const double *scale, float beta,
                      void *stream);

/* The data-fidelity dual update of Alg. 2 for every channel (one block each):
 *   z  = U^-1 v + Phi xcheck   (the transform of the extrapolated iterate)
 *   p  = projection of z onto B(y, eps_l) in the metric of U (eq.
 *        prox_definition), by forward-backward sub-iterations (Sec. 3.2):
 *        p = P_B(z), then n_sub times p <- P_B(p - gamma U (p - z)),
 *        gamma = 1 / max_j U_j, P_B the Euclidean projection
 *   v  <- U (z - p)
 *   grad += eta_l Re(Phi^dagger v)   (the data part of the aggregation)
 *   residual_l = ||y - Phi x||   (x the iterate; device FP64 [L], or null)
 * xcheck, x, grad: device FP32 [ny][nx][L]; v (in / out), y: complex FP32
 * [sum n_vis]; U: device FP32 [sum n_vis], > 0; eps, eta: device FP64 [L]. */
int fhs_data_dual_update(const fhs_data_plan *plan, const float *xcheck, const float *x, float *v, const float *y,
                         const float *U, const double *eps, const double *eta, int32_t n_sub, float *grad,
                         double *residual, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FHS_H */
