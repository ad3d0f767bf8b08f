// Internal structures shared by the host plan code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfb_device.h"

namespace pfb {

constexpr double kC0 = 299792458.0;
constexpr uint32_t kHomeBit = 0x80000000u;   // set in Rec::idx for the entry's own tile

// One bucketed visibility: coordinates local to the tile it is listed under.
//   fu, fv : grid coordinate minus the tile origin (cells); may lie outside [0, T)
//            for copies listed under a neighbouring tile the kernel straddles
//   fw     : absolute w-plane coordinate (t_w = (w - w0) / dw); 0 when flat
//   idx    : r * n_chan + c, plus kHomeBit on the copy in the tile holding (fu, fv)
template <typename R> struct Rec {
    R fu, fv, fw;
    uint32_t idx;
};

// Per-band w-stacking parameters of one gridder.
struct BandDev {
    double w0;     // w of plane 0 (wavelengths)
    double dw;     // plane spacing (wavelengths)
    double sc;     // centre of n - 1 over the image (phase split point)
    int    nw;     // w-planes of this band
    int    nj0;    // base planes (nw - W + 1), 1 when flat
};

// Spread work item: tile `tile` of band `band`, storing planes [p0, p1).
struct GridWork {
    int band, tile, p0, p1;
};
// Interpolation work item: positions [e0, e1) of one tile's home-entry list, base planes [q0, q1].
struct InterpWork {
    int band, tile, e0, e1, q0, q1;
};

// Geometry of one gridder (main w-stacked operator, or the flat PSF gridder).
struct GeomDev {
    int nx, ny;          // image
    int gx, gy;          // oversampled grid
    int T, ntx, nty;     // tiles
    int W;
    int nj0max, nwmax;   // strides
    int n_band;
    int flat;
    int offx, offy;      // pixel (nx/2, ny/2) sits at l = offx cellx, m = offy celly (a facet)
    double cellx, celly;
    double beta;
};

// Count / scatter pass inputs.
struct BucketArgs {
    GeomDev g;
    const double *uvw;
    const double *freq_dev;     // [n_chan]
    const int *chan_band_dev;   // [n_chan]
    const void *weight;         // R [n_row][n_chan]
    const uint8_t *flag;        // may be null
    const BandDev *bands;
    int64_t n_row, n_chan;
    // count pass
    int band_sel;               // >= 0: count only entries of this band, counts relative to it
    unsigned int *counts;       // [n_band * ntiles * nj0max] (one band's share when band_sel >= 0)
    unsigned int *home_counts;  // same shape: entries listed under their own (home) tile
    unsigned long long *n_active, *n_flagged, *n_bad;
    unsigned long long *n_badw;  // may be null: unflagged entries whose weight is NaN, < 0 or infinite
    // scatter pass
    unsigned long long *cursor; // [n_band * ntiles * nj0max] (starts at offsets)
    void *recs;                 // Rec<R>[n_entries]
    void *omega;                // R[n_entries]
    uint32_t *flagged;          // [n_flagged]
    unsigned long long *flag_cursor;
};

}  // namespace pfb
