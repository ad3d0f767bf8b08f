// Host-callable launchers for the gfx950 kernels (implemented in pfb_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfb_internal.h"

#include <vector>

namespace pfb {

// Records HIP events around each kernel launch of the thread that installed it.
struct Profiler {
    struct Rec {
        const char *name;   // launch expression text, e.g. "(spread_kernel<R, W, ...>)"
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    void clear();
    ~Profiler();
};
void set_thread_profiler(Profiler *p);

// All launchers return hipSuccess or the launch error; `dbl` selects float64.

hipError_t launch_count(bool dbl, const BucketArgs &a, hipStream_t s);
// Fixed device buffer for callers that cannot allocate (pfb_plan_count_static):
// its device address on the current device (looked up once per device) and size.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
hipError_t static_scratch(void **ptr);
hipError_t launch_scatter(bool dbl, const BucketArgs &a, hipStream_t s);
// home-entry list: items as for launch_sort (after it), hoffsets per bucket
hipError_t launch_home_list(bool dbl, const void *recs, const int64_t *items, int n_items, const int64_t *hoffsets,
                            uint32_t *hidx, hipStream_t s);
// home_pos[e] = home-list position of entry e's visibility (after the home list);
// vis2h is scratch of one word per visibility
hipError_t launch_home_pos(bool dbl, const void *recs, const uint32_t *hidx, int64_t n_home, int64_t n_entries,
                           uint32_t *vis2h, uint32_t *home_pos, hipStream_t s);
// Deterministic plan-time order of the entries of every bucket (pfb_sort.hip):
// items are [start, count, band, bucket] quadruples of the non-empty buckets;
// entries are ordered by (bucket, block of rb x cb base cells, visibility index);
// src -> dst (records and weights); phase (optional, FP32 complex per entry)
// receives the w-phase.  scratch holds sort_scratch_bytes(n_entries) bytes.
size_t sort_scratch_bytes(int64_t n_entries);
int sort_key_bits(int64_t n_buckets, int T, int W, int rb, int cb, int64_t n_vis);
hipError_t launch_sort(bool dbl, const void *src, const void *src_om, void *dst, void *dst_om, const int64_t *items,
                       int n_items, int64_t n_entries, int64_t n_buckets, int64_t bucket_per_band, int64_t n_vis,
                       int T, int W, int rb, int cb, const BandDev *bands, const GeomDev &geo, void *phase,
                       void *scratch, hipStream_t s);
hipError_t launch_corr2d(bool dbl, const GeomDev &g, const BandDev *bands, const double *cheb,
                         int ncheb, double xi_max, void *corr, hipStream_t s);
hipError_t launch_corr1d(bool dbl, int n, int gsize, const double *cheb, int ncheb, double xi_max,
                         void *corr, hipStream_t s);

struct SpreadLaunch {
    GeomDev g;
    const BandDev *bands;
    const GridWork *work;
    int n_work;
    const int64_t *offsets;
    const void *recs, *omega;
    const void *vis;      // VMODE 0: caller visibilities; VMODE 2: values in home-list order
    void *planes;         // [band_batch][nwmax][gx][gy]
    int band0;
    int vmode;            // 0 data, 1 unit visibilities, 2 precomputed values
    const float *absmax;  // FP32 path: device scalar, max |z| over active visibilities
    const void *phase;    // FP32 w-stacked gridder: exp(2 pi i s_c w) per entry (selects the MFMA spread)
    const uint32_t *home_pos;  // VMODE 2: per entry, the home-list position of its visibility
};
// Window of the MFMA spread for support W (4..8): footprints whose base cells lie
// in a block of rb rows x cb columns share one accumulator tile.
void mfma_window(int W, int *rb, int *cb);
// LDS bytes per block of the spread and interpolation kernels (the larger)
size_t gridder_lds_bytes(bool dbl, int W, int T, bool flat);
constexpr size_t kMaxLdsBytes = 160 * 1024;
hipError_t launch_spread(bool dbl, const SpreadLaunch &a, hipStream_t s);
// FP32 path: absmax = max over unflagged, non-zero-weight entries of |w V| (vmode 0),
// w (vmode 1) or |values| (vmode 2); partials holds >= kAbsmaxBlocks floats.
constexpr int kAbsmaxBlocks = 1024;
hipError_t launch_absmax_clear(float *absmax, hipStream_t s);
hipError_t launch_absmax(int vmode, const void *vis, const void *weight, const uint8_t *flag, int64_t n,
                         float *partials, float *absmax, hipStream_t s);

struct InterpLaunch {
    GeomDev g;
    const BandDev *bands;
    const InterpWork *work;
    int n_work;
    const int64_t *offsets;
    const void *recs, *omega;
    const void *planes;
    void *out;            // OMODE 0: visibilities; OMODE 1: values in home-list order; OMODE 2: added to
                          // the visibilities
    int band0;
    int omode;
    const void *phase;    // FP32 w-stacked gridder: exp(2 pi i (s_c w + u l0 + v m0)) per entry (else null)
    int use_phase;        // OMODE 0/2 take the visibility phase from `phase` (facets) instead of computing it
    float *absmax;        // FP32, OMODE 1: raised to max |value| x 1.0001 (cleared by the caller), or null
    const uint32_t *hidx;       // home-entry list (entry positions)
    const int64_t *hoffsets;    // per bucket: start of its home entries in hidx
};
hipError_t launch_interp(bool dbl, const InterpLaunch &a, hipStream_t s);
hipError_t launch_zero_flagged(bool dbl, const uint32_t *flagged, int64_t n, void *vis, hipStream_t s);

// FFT passes of the operator transforms.  `tw` is the forward twiddle table of
// length 2^log2_lmax.
struct XformArgs {
    GeomDev g;
    const BandDev *bands;
    int band0, n_bb;       // bands [band0, band0 + n_bb) of the batch
    const void *tw;
    int log2_lmax;
    void *planes;          // [n_bb][nwmax][gx][gy] uv planes
    void *t1;              // [n_bb][nwmax] cropped row spectra, group-major (plane_group_cols)
    const void *corr2d;    // [n_band][nx][ny] or null
    const void *corr_x, *corr_y;  // 1-D tables when corr2d is null
    const void *image_in;  // degrid input [n_band][nx][ny]
    void *image_out;       // grid output [n_band][nx][ny]
    int zero_edge;         // PSF: zero row 0 and column 0 of the output
    // [n_band][nwmax][ntx * nty] tile flags: the grid transform reads a tile of a
    // plane only where occ is set (elsewhere it is zero), the degrid transform
    // writes it only where need is set
    const uint8_t *occ, *need;
    // [n_band][nwmax][ntx]: some tile of that tile row is occ / need.  Cropped
    // rows of tile rows without occupied tiles are not written by the inverse row
    // pass and are read as zero by the grid's column pass; rows of tile rows
    // without needed tiles are neither written by the degrid's column pass nor
    // read by its row pass
    const uint8_t *occ_row, *need_row;
    // tile rows of bands [band0, band0 + n_bb) with occupied (needed) tiles, each
    // (band nwmax + plane) ntx + tile row: the inverse (forward) row pass runs on
    // their rows only
    const int32_t *occ_list, *need_list;
    int n_occ_list, n_need_list;
};
// complex values per group of the plane intermediate t1 (64 bytes)
int plane_group_cols(bool dbl);
hipError_t launch_grid_xform(bool dbl, const XformArgs &a, hipStream_t s);    // planes -> image
hipError_t launch_degrid_xform(bool dbl, const XformArgs &a, hipStream_t s);  // image -> planes

// PSF convolution machinery.
struct ConvArgs {
    int n_band, nx, ny, ldh;   // image nx x ny; per-band stride lx ldh, ldh >= ly / 2 + 1 rounded to 16
    int lx, ly;                // zero-padded grid: powers of two >= 2 nx, 2 ny (no wrap-around
                               // within the crop of the linear convolution)
    int cgc;                   // columns per group of the group-major layout (conv_group_cols)
    const void *tw;
    int log2_lmax;
    void *t1c;                 // [n_band][lx ldh] complex: row spectra, group-major
    void *psfhat;              // [n_band][lx ldh] real: PSF spectrum, group-major, even/odd split
    double *partials;          // [n_band][max_partials]
    int max_partials;
    double *scal;              // [n_band][8] device scalars
};
enum ConvIn { CONV_IN_X = 0, CONV_IN_CG_P = 1, CONV_IN_SCALED = 2 };
enum ConvOut { CONV_OUT_Y = 0, CONV_OUT_SUB = 1, CONV_OUT_CG = 2, CONV_OUT_NORM = 3, CONV_OUT_DOT = 4 };
// y = PSF * x with optional fused prologue / epilogue:
//   in  CONV_IN_CG_P : p = r + beta p (x = r, aux_in = p, written back), transform p
//       CONV_IN_SCALED: transform x * scal[S_SCALE]
//   out CONV_OUT_SUB : y = conv - aux_out          (gradient, eq. 4)
//       CONV_OUT_CG  : y = conv + sigma p, partial p . y  (CG, aux_out = p)
//       CONV_OUT_NORM: partial y . y
//       CONV_OUT_DOT : partial aux_out . y
// columns per group of the convolution's group-major layout for images of nx rows
int conv_group_cols(bool dbl, int nx);
hipError_t launch_psf_conv(bool dbl, const ConvArgs &a, const void *x, void *aux_in, void *y,
                           const void *aux_out, double sigma, int in_mode, int out_mode,
                           hipStream_t s);
// psfhat from a 2nx x 2ny PSF image (all bands)
hipError_t launch_psfhat(bool dbl, const ConvArgs &a, const void *psf_img, hipStream_t s);
int conv_partials_per_band(bool dbl, const ConvArgs &a);

// Vector kernels for CG / power iteration / FB (all bands, P = nx*ny per band).
enum VecOp {
    VEC_CG_INIT = 0,     // y = 0, r = g, p = 0; partial r.r
    VEC_CG_UPDATE = 1,   // y += alpha p; r -= alpha Ap; partial r.r
    VEC_SCALE_COPY = 2,  // y = x * scal[SCALE]
    VEC_DOT = 3,         // partial x.y
    VEC_FB_PROX = 4,     // x = max(x - gamma y - gamma lambda, 0)
    VEC_NORM = 5,        // partial x.x
};
hipError_t launch_vec(bool dbl, int op, int n_band, int64_t P, double *partials, int max_partials,
                      const double *scal, void *x, void *y, void *r, void *p, const void *ap,
                      double gamma, double lam, hipStream_t s);
int vec_partials_per_band(int64_t P);

// scalar slots in scal[b*8 + k]
enum Slot { S_RR = 0, S_ALPHA = 1, S_BETA = 2, S_PAP = 3, S_SCALE = 4, S_LAMBDA = 5, S_TMP = 6, S_RR0 = 7 };
enum ReduceOp {
    RED_SET_RR = 0,       // rr = sum; beta = 0
    RED_ALPHA = 1,        // pAp = sum; alpha = rr / pAp
    RED_BETA = 2,         // beta = sum / rr; rr = sum
    RED_INV_SQRT = 3,     // scale = 1 / sqrt(sum)
    RED_LAMBDA = 4,       // lambda = sum
    RED_STORE = 5,        // tmp = sum
};
hipError_t launch_reduce(int op, int n_band, const double *partials, int n_part, int max_partials,
                         double *scal, hipStream_t s);
hipError_t launch_copy_scalar(int n_band, const double *scal, int slot, double *dst, hipStream_t s);


// Backward step (eq. 7, regulariser of eq. 9).  A periodic orthonormal wavelet
// filter: low-pass taps h[0 .. len), len <= kMaxWaveletTaps (db6 has 12).
constexpr int kMaxWaveletTaps = 12;
struct WaveletFilter {
    double h[kMaxWaveletTaps];
    int len;
};
// One 2-D wavelet level (rows then columns) of the top-left nr x nc block in LDS
// tiles: analysis writes LL to dst_ll and the three detail quadrants to
// dst_detail; synthesis reads LL from src_ll and the details from src_detail
// (acc: add into dst).  Source and destinations must not overlap.
hipError_t launch_wavelet_analysis_level(bool dbl, const void *src, void *dst_detail, void *dst_ll,
                                         const WaveletFilter &f, int nr, int nc, int ld, int64_t img, int n_img,
                                         hipStream_t s);
hipError_t launch_wavelet_synthesis_level(bool dbl, bool acc, const void *src_ll, const void *src_detail, void *dst,
                                          const WaveletFilter &f, int nr, int nc, int ld, int64_t img, int n_img,
                                          hipStream_t s);
hipError_t launch_wave_copy(bool dbl, const void *src, void *dst, int64_t n, double scale, hipStream_t s);
hipError_t launch_wave_axpy(bool dbl, const void *x, const void *y, void *z, int64_t n, double a, hipStream_t s);   // z = x + a y
hipError_t launch_pd_primal(bool dbl, bool init, const void *z, void *x, void *d, const void *c, const void *sv,
                            void *u, int64_t n, double tau, double gamma, double sigma_u, double psi_scale, int warm,
                            hipStream_t s);
hipError_t launch_pd_dual(bool dbl, bool zero, void *v, const void *u, const void *coef, int nbasis, int n_band,
                          int64_t P, double sigma_d, double psi_scale, double lam, hipStream_t s);

}  // namespace pfb
