/*
 * pfb.h -- C ABI of the MI355X (gfx950) library for the hot path of
 * preconditioned forward-backward imaging (Bester, Repetti, Perkins, Smirnov &
 * Kenyon, "A practical preconditioner for wide-field continuum imaging of radio
 * interferometric data", ADASS XXX).
 *
 * The operators follow the paper's Section 2:
 *   V = R x + eps, eps ~ N(0, Sigma), Sigma diagonal                   (eq. 1)
 *   R : n_b real images of n_p pixels -> n_nu channels x n_d rows of complex
 *       visibilities, one imaging band per group of channels, implemented as a
 *       2-D NUFFT per band with a wide-field (w) correction           (Sec. 2)
 *   I^d = R^dagger Sigma^-1 V   (dirty image)                           (after eq. 3)
 *   R^dagger Sigma^-1 R x       (Hessian of the data fidelity)         (eq. 3)
 *   I^psf * x                   (PSF convolution, approximate Hessian) (eq. 4)
 *   U = I^psf * + sigma Id, solved by conjugate gradient              (eq. 8 and after)
 *   x_{k+1/2} = x_k - gamma U^-1 grad f(x_k), then a backward step    (eqs. 6-7)
 *
 * Conventions used throughout (the paper leaves them open):
 *   - R uses exp(-2 pi i (u l + v m + w (n - 1))) / n with (u, v, w) = uvw * f / c0
 *     in wavelengths; R^dagger uses the conjugate and returns the real part.
 *   - Pixel (i, j) of an nx x ny image sits at l = (i - nx/2) cellx,
 *     m = (j - ny/2) celly; images are [n_band][nx][ny] row-major, axis 0 = l.
 *   - Visibilities, weights and flags are [n_row][n_chan] row-major; complex
 *     values are interleaved (re, im).
 *   - weight is diag(Sigma^-1) ("natural" weighting); an entry whose flag is
 *     non-zero or whose weight is 0 is excluded everywhere and pfb_degrid
 *     writes 0 there.
 *   - The PSF is the flat (w-free, n = 1) dirty image of unit visibilities on
 *     a 2nx x 2ny grid, centred on pixel (nx, ny); row 0 and column 0 (offset
 *     -nx / -ny) are zero so that the convolution operator is exactly
 *     symmetric.  The convolution is linear (zero padded), nx x ny in and out.
 *
 * Precision: PFB_FP32 computes in float32 (images float32, visibilities
 * complex64, weights float32) with float64 only for coordinates, the
 * per-pixel correction and all CG / power-iteration scalars; PFB_FP64 computes
 * everything in float64 (images float64, visibilities complex128, weights
 * float64).  uvw and freq are always float64.
 *
 * Memory and ownership:
 *   - Every pointer documented as "device" is HIP device memory owned by the
 *     caller; the library borrows it.  uvw, weight and flag must stay valid
 *     and unchanged until pfb_plan_destroy.
 *   - The library never allocates device memory.  Plan set-up takes three
 *     calls: pfb_plan_create (validation, uvw analysis), pfb_plan_count (the
 *     counting pass, in a caller-provided scratch buffer whose size
 *     pfb_plan_count_scratch_size reports) and pfb_plan_set_workspace.  All
 *     persistent device state of a plan (visibility buckets, correction
 *     tables, twiddles, w-planes, FFT intermediates, the resident PSF
 *     spectrum, CG vectors) lives in ONE caller-provided workspace whose size
 *     pfb_plan_workspace_size reports.  pfb_plan_create and pfb_plan_count
 *     synchronise their stream (uvw and the bucket counts are read on the
 *     host); so does pfb_precond_solve with tol > 0; nothing else does.
 *   - Operator calls are asynchronous on the stream they are given and contain
 *     no host synchronisation.  A plan is not thread-safe; calls on one plan
 *     must be serialised on one stream.  Distinct plans are independent.
 *
 * Errors: every entry point returns a pfb_status; 0 is success.  A non-zero
 * status leaves outputs unspecified and pfb_last_error() returns a
 * thread-local message.  Device faults surface at the next synchronising call.
 */
#ifndef PFB_H
#define PFB_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int pfb_status;
#define PFB_OK            0
#define PFB_EINVAL       -1   /* bad argument: shape, null pointer, odd image side, NaN uvw,
                                 a pixel with l^2 + m^2 >= 1, unsupported support/oversampling */
#define PFB_ENOMEM       -2   /* workspace missing or smaller than required */
#define PFB_EHIP         -3   /* a HIP runtime call or kernel launch failed */
#define PFB_EUNSUPPORTED -4   /* valid request the library does not implement */
#define PFB_ESTATE       -5   /* call order: e.g. psf_conv before the PSF spectrum exists */

#define PFB_FP32 0
#define PFB_FP64 1

/* pfb_grid modes */
#define PFB_GRID_DIRTY 0   /* image = R^dagger Sigma^-1 V, [n_band][nx][ny]                     */
#define PFB_GRID_PSF   1   /* V := 1, flat: image = PSF, [n_band][2nx][2ny]; also makes the
                              resident PSF spectrum used by pfb_psf_conv / solve / fb_step   */

typedef struct pfb_plan pfb_plan;

/* The imaging problem (eq. 1 with the shapes of Section 2). */
typedef struct {
    int64_t        n_row;      /* n_d: rows (baseline x time samples)                       */
    int64_t        n_chan;     /* n_nu: channels                                            */
    int32_t        n_band;     /* n_b: imaging bands                                        */
    const int32_t *chan_band;  /* HOST int32[n_chan]: band of each channel, in [0, n_band)   */
    const double  *freq;       /* HOST float64[n_chan]: channel frequency, Hz (> 0)          */
    const double  *uvw;        /* DEVICE float64[n_row][3]: baseline coordinates, metres     */
    const void    *weight;     /* DEVICE [n_row][n_chan] diag(Sigma^-1), float32 for PFB_FP32,
                                  float64 for PFB_FP64; entries must be >= 0                  */
    const uint8_t *flag;       /* DEVICE uint8[n_row][n_chan] (non-zero = flagged) or NULL    */
    int32_t        nx, ny;     /* image side lengths, even, >= 16                           */
    double         cellx;      /* pixel size along l, radians                               */
    double         celly;      /* pixel size along m, radians                               */
    int32_t        offx, offy; /* facet offset in pixels: pixel (nx/2, ny/2) of this image sits at
                                  l = offx cellx, m = offy celly (0, 0: centred on the phase
                                  centre).  Non-zero offsets: FP32, not flat                   */
} pfb_problem;

/* Accuracy / tiling choices.  Zero fields take the defaults given. */
typedef struct {
    int32_t precision;    /* PFB_FP32 (default) or PFB_FP64                                  */
    int32_t support;      /* ES kernel support W in cells: default 7 (FP32), 13 (FP64);
                             FP32 accepts 4..8, FP64 accepts 9..16                           */
    double  oversample;   /* grid oversampling sigma; only 2.0 is implemented (default)     */
    int32_t tile;         /* uv tile side T (power of two, 8..64); default 32 FP32, 8 FP64   */
    int32_t flat;         /* 1: drop the w term and the 1/n factor from R (w = 0, n = 1)     */
    int32_t band_batch;   /* bands whose w-planes are resident at once; default n_band       */
    int32_t chunk;        /* bucket entries per work item before a tile is split (>= 64);
                             default max(4096, entries / compute units of the device)       */
    double  epsilon;      /* requested relative accuracy of grid / degrid (rel-l2); when
                             support is 0 and epsilon > 0 the support is the smallest W whose
                             tabulated error of the 3-D ES product kernel at sigma = 2 plus
                             the arithmetic's rounding floor is <= epsilon (FP32: W 4..8,
                             reach ~2.3e-6; FP64: W 9..16, reach ~1.5e-14); a smaller
                             epsilon than the precision reaches is PFB_EINVAL.  0: the
                             default support.                                               */
    int32_t reserved[6];
} pfb_options;

/* Read-only description of a created plan. */
typedef struct {
    int32_t grid_x, grid_y;        /* oversampled uv grid of the operator                   */
    int32_t psf_grid_x, psf_grid_y;/* oversampled grid of the 2nx x 2ny PSF                 */
    int32_t support, tile;
    int32_t n_wplanes_max;         /* largest number of w-planes over bands                 */
    int32_t band_batch;
    int64_t n_vis_active;          /* unflagged, non-zero-weight visibilities               */
    int64_t n_entries;             /* bucket entries incl. copies for tile-straddling kernels */
    int64_t n_psf_entries;
    double  s_min;                 /* min over pixels of n - 1                              */
    double  es_beta;               /* ES kernel shape parameter                             */
    int64_t workspace_bytes;
    /* occupancy of the operator's (band, w-plane, uv tile) cells, summed over bands
       and their own planes: the spread writes occ_tiles of them (the rest is zero
       and is not read by the grid transform), the degrid transform writes the
       need_tiles the interpolation may read; *_tile_rows count the (band, plane,
       tile row) triples with at least one such tile                           */
    int64_t n_wplanes_total;       /* sum over bands of their w-planes                      */
    int64_t occ_tiles, occ_tile_rows, need_tiles, need_tile_rows;
    double  s_max;                 /* max over pixels of n - 1 (0 when the image holds the
                                      phase centre)                                          */
} pfb_plan_info;

/* Creates a plan: validates the problem and analyses uvw (copied to the host on
 * `stream`, which is synchronised) to fix the grids and w-planes of every band
 * (Section 2: R per band).  Allocates no device memory.  On success *plan must be
 * released with pfb_plan_destroy; pfb_plan_count comes next. */
pfb_status pfb_plan_create(pfb_plan **plan, const pfb_problem *prob, const pfb_options *opt,
                           hipStream_t stream);

/* Bytes of the device scratch buffer pfb_plan_count needs: one band's counters per
 * (uv tile, w base plane) of the operator and the PSF gridders plus small tables
 * (bands are counted one after another). */
pfb_status pfb_plan_count_scratch_size(const pfb_plan *plan, size_t *bytes);

/* Counting pass: the visibilities of every band are counted per (uv tile, w base
 * plane) in `scratch` (DEVICE, >= pfb_plan_count_scratch_size bytes, 256-byte
 * aligned, borrowed only for this call: it may be reused once the call returns),
 * then the work lists and the workspace layout are fixed on the host.
 * Synchronises `stream`.  Fails with PFB_EINVAL if an unflagged weight is NaN,
 * negative or infinite.  Once per plan (PFB_ESTATE on a second call). */
pfb_status pfb_plan_count(pfb_plan *plan, void *scratch, size_t bytes, hipStream_t stream);

/* pfb_plan_count without a scratch argument, for callers that cannot allocate
 * device memory at all: the counting pass runs in a fixed 64 MiB buffer that the
 * library holds on every device it runs on until the process ends (allocated when
 * the library's code is loaded, not by this call, which allocates nothing).  A plan
 * whose pfb_plan_count_scratch_size exceeds 64 MiB gets PFB_ENOMEM.  The buffer is
 * shared by every call on a device and cleared by each call where it must start at
 * zero; calls that overlap on one device (other threads, other streams) race and
 * must be serialised by the caller.  Otherwise as pfb_plan_count. */
pfb_status pfb_plan_count_static(pfb_plan *plan, hipStream_t stream);

/* Bytes of device workspace the plan needs (256-byte aligned pointer expected);
 * valid after pfb_plan_count. */
pfb_status pfb_plan_workspace_size(const pfb_plan *plan, size_t *bytes);

/* Hands the plan its workspace and enqueues on `stream` the one-off set-up
 * inside it: visibility buckets, correction and twiddle tables.  `dev` must
 * stay valid until pfb_plan_destroy.  Must precede every operator call. */
pfb_status pfb_plan_set_workspace(pfb_plan *plan, void *dev, size_t bytes, hipStream_t stream);

pfb_status pfb_plan_get_info(const pfb_plan *plan, pfb_plan_info *info);

/* Frees host memory of the plan (not the caller's workspace). NULL is accepted. */
pfb_status pfb_plan_destroy(pfb_plan *plan);

/* Dirty image I^d = R^dagger Sigma^-1 V (Section 2, after eq. 3).
 *   vis   DEVICE complex [n_row][n_chan] (ignored, may be NULL, in PFB_GRID_PSF mode)
 *   image DEVICE real [n_band][nx][ny] (DIRTY) or [n_band][2nx][2ny] (PSF; may be NULL
 *         when only the resident spectrum is wanted). */
pfb_status pfb_grid(pfb_plan *plan, const void *vis, void *image, int mode, hipStream_t stream);

/* Model visibilities V = R x (eq. 1 without noise; not weighted).
 *   image DEVICE real [n_band][nx][ny];  vis DEVICE complex [n_row][n_chan] (fully written;
 *   flagged / zero-weight entries get 0). */
pfb_status pfb_degrid(pfb_plan *plan, const void *image, void *vis, hipStream_t stream);

/* V += R x: as pfb_degrid, but the model visibilities of x are added to vis, and
 * flagged / zero-weight entries are left as they are.  With facet plans (pfb_problem
 * offx, offy) that share one set of visibilities, the model visibilities of a whole
 * image are the sum over its facets (Section 2: R is linear in x). */
pfb_status pfb_degrid_add(pfb_plan *plan, const void *image, void *vis, hipStream_t stream);

/* y = R^dagger Sigma^-1 R x (eq. 3), x and y DEVICE real [n_band][nx][ny]; x != y. */
pfb_status pfb_hessian(pfb_plan *plan, const void *x, void *y, hipStream_t stream);

/* y = I^psf * x (eq. 4), linear convolution with the resident PSF of each band.
 * x, y DEVICE real [n_band][nx][ny]; x may equal y.  Needs pfb_grid(PFB_GRID_PSF) first. */
pfb_status pfb_psf_conv(pfb_plan *plan, const void *x, void *y, hipStream_t stream);

/* Solves (I^psf * + sigma Id) y = g by at most `iters` conjugate-gradient steps from
 * y = 0 (eq. 8 and the sentence after it); every band independently.  Inner products
 * and step lengths are float64 on the device.  g, y DEVICE real [n_band][nx][ny], g != y.
 * tol = 0: exactly `iters` steps, no host synchronisation (graph-capturable).
 * tol > 0: the loop stops after the first step at which every band has
 * ||r||_2 <= tol ||g||_2; the residuals are read on the host after every step, so the
 * call synchronises `stream` and is refused (PFB_ESTATE) while the stream is capturing.
 * dev_resid: NULL or DEVICE float64[n_band], receives the final squared residual norm. */
pfb_status pfb_precond_solve(pfb_plan *plan, const void *g, void *y, double sigma, int iters,
                             double tol, double *dev_resid, hipStream_t stream);

/* Power iteration for the largest eigenvalue of op (0 = I^psf *, 1 = R^dagger Sigma^-1 R),
 * per band: v <- A v / ||A v|| `iters` times from v0, then lambda = v^T A v.  float64
 * norms.  v0 DEVICE real [n_band][nx][ny] (not modified); dev_lambda DEVICE float64[n_band]. */
pfb_status pfb_power_iteration(pfb_plan *plan, int op, const void *v0, int iters,
                               double *dev_lambda, hipStream_t stream);

/* One preconditioned forward-backward step with the PSF-approximate gradient (eq. 4):
 *   g = I^psf * x - I^d;  y = U^-1 g by `cg_iters` CG steps, U = I^psf * + sigma Id (eq. 8);
 *   x <- max(x - gamma y - gamma lambda, 0), the Euclidean prox of
 *   gamma (lambda ||.||_1 + positivity) standing in for eq. (7).
 * dirty, x DEVICE real [n_band][nx][ny]; x is updated in place. */
pfb_status pfb_fb_step(pfb_plan *plan, const void *dirty, void *x, double sigma, double gamma,
                       double lambda, int cg_iters, hipStream_t stream);

/* ---- Backward step of the paper: eq. (7) with the regulariser of eq. (9) ----
 * r(x) = lambda ||Psi^dagger x||_{2,1} + positivity.  Psi is the dictionary of the
 * Dirac basis and the first nbasis - 1 Daubechies wavelet bases (db1, db2, ...;
 * the paper uses nbasis = 7), each a periodic orthonormal 2-D transform of
 * `levels` levels (Mallat layout), scaled by 1/sqrt(nbasis) so that
 * Psi Psi^dagger = Id.  The l2 norm runs over the bands of one basis coefficient,
 * the l1 sum over bases and coefficients.  Daubechies filters are computed from
 * their defining polynomial (minimum phase, coefficients summing to sqrt 2).
 * Coefficient arrays are DEVICE real [nbasis][n_band][nx][ny] in the plan's
 * precision; nx and ny must be multiples of 2^levels, 1 <= nbasis <= 7,
 * 1 <= levels <= 16.  ws is a DEVICE buffer of at least pfb_prox_workspace_size
 * bytes owned by the caller; it holds the dual variable between calls. */
pfb_status pfb_prox_workspace_size(const pfb_plan *plan, int nbasis, size_t *bytes);

/* coeffs = Psi^dagger x.  x DEVICE real [n_band][nx][ny]. */
pfb_status pfb_wavelet_analysis(pfb_plan *plan, const void *x, void *coeffs, void *ws, size_t ws_bytes,
                                int nbasis, int levels, hipStream_t stream);

/* x = Psi coeffs (the adjoint of pfb_wavelet_analysis and, for a tight frame, its
 * left inverse). */
pfb_status pfb_wavelet_synthesis(pfb_plan *plan, const void *coeffs, void *x, void *ws, size_t ws_bytes,
                                 int nbasis, int levels, hipStream_t stream);

/* x = prox^U_{gamma r}(z) of eq. (7), U = I^psf * + sigma Id, by `iters` iterations of
 * the primal-dual algorithm of Condat (2013) named after eq. (8):
 *   x~ = max(x - tau (U (x - z) / gamma + Psi v), 0)
 *   v  = P_lambda(v + sigma_d Psi^dagger (2 x~ - x)),  x = x~
 * where P_lambda scales every band vector of v onto the l2 ball of radius lambda,
 * beta = (unorm + sigma) / gamma, sigma_d = beta, tau = 0.99 / (beta / 2 + sigma_d).
 * unorm >= ||I^psf *|| (e.g. pfb_power_iteration with a margin).  warm = 0 starts
 * from x = max(z, 0), v = 0; warm != 0 continues from the x passed in and the v
 * left in ws by the previous call, which must have used the same plan, ws and
 * nbasis (the dual is not checked).  z, x DEVICE real [n_band][nx][ny], z != x;
 * the plan's PSF spectrum must exist.  Calls on one ws must not overlap. */
pfb_status pfb_prox_solve(pfb_plan *plan, const void *z, void *x, void *ws, size_t ws_bytes, int nbasis,
                          int levels, double lambda, double gamma, double sigma, double unorm, int iters,
                          int warm, hipStream_t stream);

/* One forward-backward step of the paper (eqs. 6-7 with the regulariser of eq. 9):
 *   z = x - gamma U^-1 (I^psf * x - I^d), U^-1 by `cg_iters` CG steps (as pfb_fb_step);
 *   x = prox^U_{gamma r}(z) by `pd_iters` iterations of pfb_prox_solve (warm as there:
 *   warm != 0 starts the primal-dual iteration from the x passed in and the dual
 *   variable kept in ws).  ws as for pfb_prox_solve (the same size query); dirty, x
 *   DEVICE real [n_band][nx][ny]; x is updated in place. */
pfb_status pfb_fb_step_wavelet(pfb_plan *plan, const void *dirty, void *x, void *ws, size_t ws_bytes, int nbasis,
                               int levels, double sigma, double gamma, double lambda, double unorm, int cg_iters,
                               int pd_iters, int warm, hipStream_t stream);

/* pfb-clean iterations (Sec. 2): `n_major` preconditioned forward-backward steps with
 * the exact gradient, each one Hessian application (eq. 3):
 *   g = R^dagger Sigma^-1 R x - I^d;  z = x - gamma U^-1 g (`cg_iters` CG steps, eq. 6,
 *   U = I^psf * + sigma Id, eq. 8);  x = prox^U_{gamma r}(z) (eq. 7, prior of eq. 9,
 *   `pd_iters` primal-dual steps, warm-started from the previous step after the first).
 * Arguments as for pfb_fb_step_wavelet; x DEVICE real [n_band][nx][ny] in/out. */
pfb_status pfb_clean(pfb_plan *plan, const void *dirty, void *x, void *ws, size_t ws_bytes, int nbasis, int levels,
                     double sigma, double gamma, double lambda, double unorm, int cg_iters, int pd_iters,
                     int n_major, hipStream_t stream);

/* hipGraph capture of forward-backward iterations (for launch-bound loops).
 * Captures `n_steps` consecutive pfb_fb_step(plan, dirty, x, sigma, gamma, lambda,
 * cg_iters) calls into one instantiated HIP graph.  `stream` must be a
 * non-default stream; it is used only during capture.  The graph reads and
 * writes the same device buffers on every launch (x is updated in place) and
 * contains no memset or host work; the plan's PSF spectrum must exist.  The
 * graph borrows the plan, its workspace, dirty and x: keep them alive and do not
 * run other calls on this plan concurrently with a launch. */
typedef struct pfb_graph pfb_graph;
pfb_status pfb_fb_graph_create(pfb_plan *plan, const void *dirty, void *x, double sigma, double gamma,
                               double lambda, int cg_iters, int n_steps, hipStream_t stream,
                               pfb_graph **graph);
/* Launches the captured iterations on `stream` (asynchronous). */
pfb_status pfb_graph_launch(pfb_graph *graph, hipStream_t stream);
/* Frees the graph (NULL accepted). */
pfb_status pfb_graph_destroy(pfb_graph *graph);

/* Diagnostics: while enabled, every kernel that an operator call on this plan
 * launches is bracketed by HIP events recorded on that call's stream.  on != 0
 * discards earlier records and starts recording; on == 0 stops. */
pfb_status pfb_profile_enable(pfb_plan *plan, int on);

/* Synchronises on the recorded events and writes one line per kernel,
 * "name launches total_ms\n", into buf (NUL-terminated, truncated to len). */
pfb_status pfb_profile_report(pfb_plan *plan, char *buf, size_t len);

/* Thread-local text of the last non-OK status (never NULL). */
const char *pfb_last_error(void);

/* Library version string. */
const char *pfb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PFB_H */
