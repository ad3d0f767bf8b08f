// gfx950 kernels of the pfb-clean hot path:
//   * bucketing of visibilities into (band, uv tile, w base plane) buckets
//   * ES-kernel gridding with owner-computes uv tiles (no global atomics)
//   * ES-kernel degridding with a sliding window of w-planes in LDS
//   * the 2-D FFT passes (LDS radix-8 rows; single-pass columns that split the
//     zero-padded transforms into two halves and loop over the w-planes) with
//     the w-phase, cropping, padding and grid correction fused into them
//   * PSF convolution by zero-padded FFT and the CG / power-iteration kernels
#include <type_traits>
#include <utility>

#include "pfb_kernels.h"
#include <limits>
#include <mutex>

namespace pfb {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <int LO, int HI, class F>
static hipError_t dispatch_int(int v, F &&f) {
    if constexpr (LO <= HI) {
        if (v == LO) return f(std::integral_constant<int, LO>{});
        return dispatch_int<LO + 1, HI>(v, std::forward<F>(f));
    } else {
        return hipErrorInvalidValue;
    }
}

template <class K>
static hipError_t set_lds(K kernel, size_t bytes) {
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Optional per-launch timing: HIP events recorded on the launch stream around
// every kernel while a profiler is installed for the calling thread.
thread_local Profiler *t_prof = nullptr;
void set_thread_profiler(Profiler *p) { t_prof = p; }

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
void Profiler::clear() {
    for (auto &r : recs) {
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
}
Profiler::~Profiler() {
    clear();
    for (auto e : pool) (void)hipEventDestroy(e);
}

#define PFB_LAUNCH(kernel, grid, lds, stream, ...) PFB_LAUNCH_NT(kernel, grid, kThreads, lds, stream, __VA_ARGS__)

#define PFB_LAUNCH_NT(kernel, grid, nthreads, lds, stream, ...)                      \
    do {                                                                             \
        hipError_t _e = set_lds(kernel, (lds));                                      \
        if (_e != hipSuccess) return _e;                                             \
        hipEvent_t _ea = nullptr;                                                    \
        if (t_prof) {                                                                \
            _ea = t_prof->get();                                                     \
            (void)hipEventRecord(_ea, stream);                                       \
        }                                                                            \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(nthreads), (lds), stream,        \
                           __VA_ARGS__);                                             \
        _e = hipGetLastError();                                                      \
        if (_e != hipSuccess) return _e;                                             \
        if (t_prof) {                                                                \
            hipEvent_t _eb = t_prof->get();                                          \
            (void)hipEventRecord(_eb, stream);                                       \
            t_prof->recs.push_back({#kernel, _ea, _eb});                             \
        }                                                                            \
    } while (0)

__device__ __forceinline__ int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }

// exp(-2 pi i t / 16), t = 0 .. 7: w^(t N / 8) for w = exp(-2 pi i / 2N), the
// factor between the eight inputs of an outermost radix-8 butterfly (t a constant
// once the loop over t is unrolled)
template <typename R> __device__ __forceinline__ cplx<R> root16(int t) {
    const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173), h = R(0.70710678118654752440);
    switch (t) {
        case 0: return cplx<R>{R(1), R(0)};
        case 1: return cplx<R>{c1, -s1};
        case 2: return cplx<R>{h, -h};
        case 3: return cplx<R>{s1, -c1};
        case 4: return cplx<R>{R(0), R(-1)};
        case 5: return cplx<R>{-s1, -c1};
        case 6: return cplx<R>{-h, -h};
        default: return cplx<R>{-c1, -s1};
    }
}
__device__ __forceinline__ int wrapi(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

// block-wide FP64 sum over NT threads; result valid in thread 0
template <int NT = kThreads> __device__ double block_sum(double v, double *red) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wid = threadIdx.x >> 6, ln = threadIdx.x & 63;
    __syncthreads();
    if (ln == 0) red[wid] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) t += red[k];
    return t;
}

// ---------------------------------------------------------------------------
// bucketing
// ---------------------------------------------------------------------------

template <typename R>
struct Keys {
    R fu, fv, fw;
    int tu, tv, j0, ou_lo, ou_hi, ov_lo, ov_hi;
};

// Grid coordinates of one visibility and the tiles its W x W footprint touches.
// The local coordinates are rounded to R first so that the kernels, which
// recompute the footprint from them, agree exactly with the bucket keys.
template <typename R, bool FLAT>
__device__ __forceinline__ bool vis_keys(const GeomDev &g, const BandDev &bd, double um, double vm,
                                         double wm, double f, Keys<R> &k) {
    const double s = f / kC0;
    double tu = um * s * g.cellx * (double)g.gx;
    double tv = vm * s * g.celly * (double)g.gy;
    tu -= (double)g.gx * floor(tu / (double)g.gx);
    tv -= (double)g.gy * floor(tv / (double)g.gy);
    if (tu >= (double)g.gx) tu -= (double)g.gx;
    if (tv >= (double)g.gy) tv -= (double)g.gy;
    k.tu = min((int)(tu / g.T), g.ntx - 1);
    k.tv = min((int)(tv / g.T), g.nty - 1);
    k.fu = (R)(tu - (double)k.tu * g.T);
    k.fv = (R)(tv - (double)k.tv * g.T);
    const R hw = R(0.5) * (R)g.W;
    const int i0 = (int)dev_floor(k.fu - hw) + 1;
    const int j0 = (int)dev_floor(k.fv - hw) + 1;
    // tiles (relative to the home tile) overlapped by cells [i0, i0 + W)
    k.ou_lo = floordiv(i0, g.T);
    k.ou_hi = floordiv(i0 + g.W - 1, g.T);
    k.ov_lo = floordiv(j0, g.T);
    k.ov_hi = floordiv(j0 + g.W - 1, g.T);
    if (FLAT) {
        k.fw = R(0);
        k.j0 = 0;
        return true;
    }
    const double tw = (wm * s - bd.w0) / bd.dw;
    k.fw = (R)tw;
    k.j0 = (int)dev_floor(k.fw - hw) + 1;
    return k.j0 >= 0 && k.j0 < bd.nj0;
}

template <typename R, bool FLAT, bool SCATTER>
__global__ __launch_bounds__(kThreads) void bucket_kernel(BucketArgs a) {
    const int64_t total = a.n_row * a.n_chan;
    const int ntiles = a.g.ntx * a.g.nty;
    const R *wt = reinterpret_cast<const R *>(a.weight);
    unsigned long long n_act = 0, n_flag = 0, n_bad = 0, n_badw = 0;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < total; base += (int64_t)gridDim.x * kThreads) {
        const int64_t e = base + threadIdx.x;
        bool valid = e < total;
        bool flagged = false;
        R w = R(0);
        int64_t r = 0;
        int c = 0;
        if (valid) {
            r = e / a.n_chan;
            c = (int)(e - r * a.n_chan);
        }
        if (!SCATTER && valid && a.band_sel >= 0 && a.chan_band_dev[c] != a.band_sel) valid = false;
        if (valid) {
            w = wt[e];
            const bool fl = a.flag && a.flag[e];
            flagged = fl || !(w > R(0));
            // the weights are diag(Sigma^-1): a NaN, negative or infinite weight of an
            // unflagged entry is an input error (counted; the plan is refused)
            if (!SCATTER && !fl && !(w >= R(0) && w <= std::numeric_limits<R>::max())) ++n_badw;
        }
        if (SCATTER && a.flagged) {
            // wave-aggregated append of flagged indices
            const unsigned long long m = __ballot(valid && flagged);
            if (m) {
                const int leader = __ffsll((long long)m) - 1;
                unsigned long long b0 = 0;
                if (lane == leader) b0 = atomicAdd(a.flag_cursor, (unsigned long long)__popcll(m));
                b0 = __shfl(b0, leader, 64);
                if (valid && flagged) {
                    const int rank = __popcll(m & ((1ull << lane) - 1ull));
                    a.flagged[b0 + rank] = (uint32_t)e;
                }
            }
        }
        if (!valid) continue;
        if (flagged) {
            ++n_flag;
            continue;
        }
        const int b = a.chan_band_dev[c];
        const BandDev bd = a.bands[b];
        Keys<R> k;
        const bool ok = vis_keys<R, FLAT>(a.g, bd, a.uvw[3 * r], a.uvw[3 * r + 1], a.uvw[3 * r + 2],
                                          a.freq_dev[c], k);
        if (!ok) {
            ++n_bad;
            continue;
        }
        ++n_act;
        for (int ou = k.ou_lo; ou <= k.ou_hi; ++ou) {
            for (int ov = k.ov_lo; ov <= k.ov_hi; ++ov) {
                const int tile = wrapi(k.tu + ou, a.g.ntx) * a.g.nty + wrapi(k.tv + ov, a.g.nty);
                const int64_t key = ((int64_t)b * ntiles + tile) * a.g.nj0max + k.j0;
                if (!SCATTER) {
                    const int64_t kc = key - (a.band_sel >= 0 ? (int64_t)a.band_sel * ntiles * a.g.nj0max : 0);
                    atomicAdd(a.counts + kc, 1u);
                    if (ou == 0 && ov == 0) atomicAdd(a.home_counts + kc, 1u);
                } else {
                    const unsigned long long pos = atomicAdd(a.cursor + key, 1ull);
                    Rec<R> rec;
                    rec.fu = k.fu - (R)(ou * a.g.T);
                    rec.fv = k.fv - (R)(ov * a.g.T);
                    rec.fw = k.fw;
                    rec.idx = (uint32_t)e | ((ou == 0 && ov == 0) ? kHomeBit : 0u);
                    reinterpret_cast<Rec<R> *>(a.recs)[pos] = rec;
                    reinterpret_cast<R *>(a.omega)[pos] = w;
                }
            }
        }
    }
    if (!SCATTER) {
        if (n_act) atomicAdd(a.n_active, n_act);
        if (n_flag) atomicAdd(a.n_flagged, n_flag);
        if (n_bad) atomicAdd(a.n_bad, n_bad);
        if (n_badw && a.n_badw) atomicAdd(a.n_badw, n_badw);
    }
}

template <bool SCATTER>
static hipError_t launch_bucket(bool dbl, const BucketArgs &a, hipStream_t s) {
    const int64_t total = a.n_row * a.n_chan;
    int64_t nb = (total + kThreads - 1) / kThreads;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    if (dbl) {
        if (a.g.flat) PFB_LAUNCH((bucket_kernel<double, true, SCATTER>), nb, 0, s, a);
        else PFB_LAUNCH((bucket_kernel<double, false, SCATTER>), nb, 0, s, a);
    } else {
        if (a.g.flat) PFB_LAUNCH((bucket_kernel<float, true, SCATTER>), nb, 0, s, a);
        else PFB_LAUNCH((bucket_kernel<float, false, SCATTER>), nb, 0, s, a);
    }
    return hipSuccess;
}
hipError_t launch_count(bool dbl, const BucketArgs &a, hipStream_t s) { return launch_bucket<false>(dbl, a, s); }

// The counting scratch of pfb_plan_count_static.  In host code `scratch` names a
// host-side stand-in, never device memory: its device address is looked up per
// device with hipGetSymbolAddress (each device holds its own copy) and only that
// address reaches kernels, memsets and copies.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}
hipError_t launch_scatter(bool dbl, const BucketArgs &a, hipStream_t s) { return launch_bucket<true>(dbl, a, s); }

// Home-entry list of every bucket (plan time): the positions of the entries
// that carry kHomeBit, in bucket order (a stable, deterministic compaction),
// at hoffsets[bucket].  The interpolation walks this list, so it neither
// visits nor balances its work over the copies listed for neighbouring tiles.
template <typename R>
__global__ __launch_bounds__(kThreads) void home_list_kernel(const Rec<R> *recs, const int64_t *items,
                                                             const int64_t *hoffsets, uint32_t *hidx) {
    __shared__ unsigned wcount[kThreads / 64];
    const int64_t start = items[4 * blockIdx.x], n = items[4 * blockIdx.x + 1], key = items[4 * blockIdx.x + 3];
    int64_t out = hoffsets[key];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t base = 0; base < n; base += kThreads) {
        const int64_t e = base + threadIdx.x;
        const bool home = e < n && (recs[start + e].idx & kHomeBit);
        const unsigned long long m = __ballot(home);
        if (lane == 0) wcount[wv] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned before = 0, total = 0;
        for (int k = 0; k < kThreads / 64; ++k) {
            if (k < wv) before += wcount[k];
            total += wcount[k];
        }
        if (home) hidx[out + before + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)(start + e);
        out += total;
        __syncthreads();
    }
}
// home_pos[e]: home-list position of the home entry of entry e's visibility
// (vis2h: visibility index -> home-list position, n_vis words of scratch)
template <typename R>
__global__ __launch_bounds__(kThreads) void vis_home_kernel(const Rec<R> *recs, const uint32_t *hidx, int64_t n_home,
                                                            uint32_t *vis2h) {
    for (int64_t h = (int64_t)blockIdx.x * kThreads + threadIdx.x; h < n_home; h += (int64_t)gridDim.x * kThreads)
        vis2h[recs[hidx[h]].idx & ~kHomeBit] = (uint32_t)h;
}
template <typename R>
__global__ __launch_bounds__(kThreads) void home_pos_kernel(const Rec<R> *recs, int64_t n_entries,
                                                            const uint32_t *vis2h, uint32_t *home_pos) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n_entries; e += (int64_t)gridDim.x * kThreads)
        home_pos[e] = vis2h[recs[e].idx & ~kHomeBit];
}
hipError_t launch_home_pos(bool dbl, const void *recs, const uint32_t *hidx, int64_t n_home, int64_t n_entries,
                           uint32_t *vis2h, uint32_t *home_pos, hipStream_t s) {
    if (n_entries <= 0) return hipSuccess;
    const int nb = (int)std::min<int64_t>(4096, (std::max(n_home, n_entries) + kThreads - 1) / kThreads);
    if (dbl) {
        if (n_home > 0) PFB_LAUNCH(vis_home_kernel<double>, nb, 0, s, (const Rec<double> *)recs, hidx, n_home, vis2h);
        PFB_LAUNCH(home_pos_kernel<double>, nb, 0, s, (const Rec<double> *)recs, n_entries, vis2h, home_pos);
    } else {
        if (n_home > 0) PFB_LAUNCH(vis_home_kernel<float>, nb, 0, s, (const Rec<float> *)recs, hidx, n_home, vis2h);
        PFB_LAUNCH(home_pos_kernel<float>, nb, 0, s, (const Rec<float> *)recs, n_entries, vis2h, home_pos);
    }
    return hipSuccess;
}
hipError_t launch_home_list(bool dbl, const void *recs, const int64_t *items, int n_items, const int64_t *hoffsets,
                            uint32_t *hidx, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (dbl) PFB_LAUNCH(home_list_kernel<double>, n_items, 0, s, (const Rec<double> *)recs, items, hoffsets, hidx);
    else PFB_LAUNCH(home_list_kernel<float>, n_items, 0, s, (const Rec<float> *)recs, items, hoffsets, hidx);
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// grid correction
// ---------------------------------------------------------------------------

// Fourier transform of the ES kernel, psi_hat(xi) for |xi| <= xi_max, from its
// Chebyshev expansion in y = 2 (xi / xi_max)^2 - 1 (the transform is even).
__device__ double psihat_eval(const double *c, int n, double xi, double xi_max) {
    const double t = xi / xi_max;
    const double y = 2.0 * t * t - 1.0;
    double b1 = 0, b2 = 0;
    for (int k = n - 1; k >= 1; --k) {
        const double b0 = c[k] + 2.0 * y * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + y * b1 - b2;
}

// corr[b][i][j] = 1 / (psi_hat_u psi_hat_v [psi_hat_w(dw (s - sc)) n])
template <typename R>
__global__ __launch_bounds__(kThreads) void corr2d_kernel(GeomDev g, const BandDev *bands, const double *cheb,
                                                          int ncheb, double xi_max, R *corr) {
    const int64_t P = (int64_t)g.nx * g.ny;
    const int64_t total = P * g.n_band;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
        const int b = (int)(e / P);
        const int64_t p = e - (int64_t)b * P;
        const int i = (int)(p / g.ny), j = (int)(p - (int64_t)i * g.ny);
        const double qi = i - g.nx / 2, qj = j - g.ny / 2;
        double c = psihat_eval(cheb, ncheb, qi / g.gx, xi_max) * psihat_eval(cheb, ncheb, qj / g.gy, xi_max);
        if (!g.flat) {
            const double l = (qi + g.offx) * g.cellx, m = (qj + g.offy) * g.celly;
            const double r2 = l * l + m * m;
            const double n = sqrt(1.0 - r2);
            const double sm1 = -r2 / (1.0 + n);
            const BandDev bd = bands[b];
            c *= psihat_eval(cheb, ncheb, bd.dw * (sm1 - bd.sc), xi_max) * n;
        }
        corr[e] = (R)(1.0 / c);
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void corr1d_kernel(int n, int gsize, const double *cheb, int ncheb,
                                                          double xi_max, R *corr) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) corr[i] = (R)(1.0 / psihat_eval(cheb, ncheb, (double)(i - n / 2) / gsize, xi_max));
}

hipError_t launch_corr2d(bool dbl, const GeomDev &g, const BandDev *bands, const double *cheb, int ncheb,
                         double xi_max, void *corr, hipStream_t s) {
    int64_t nb = ((int64_t)g.nx * g.ny * g.n_band + kThreads - 1) / kThreads;
    if (nb > 65536) nb = 65536;
    if (dbl) PFB_LAUNCH(corr2d_kernel<double>, nb, 0, s, g, bands, cheb, ncheb, xi_max, (double *)corr);
    else PFB_LAUNCH(corr2d_kernel<float>, nb, 0, s, g, bands, cheb, ncheb, xi_max, (float *)corr);
    return hipSuccess;
}
hipError_t launch_corr1d(bool dbl, int n, int gsize, const double *cheb, int ncheb, double xi_max, void *corr,
                         hipStream_t s) {
    const int nb = (n + kThreads - 1) / kThreads;
    if (dbl) PFB_LAUNCH(corr1d_kernel<double>, nb, 0, s, n, gsize, cheb, ncheb, xi_max, (double *)corr);
    else PFB_LAUNCH(corr1d_kernel<float>, nb, 0, s, n, gsize, cheb, ncheb, xi_max, (float *)corr);
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// gridding: owner-computes uv tiles, sliding ring of W w-planes in LDS
// ---------------------------------------------------------------------------
// Each work item owns the T x T core cells of one uv tile for planes [p0, p1).
// Its bucket lists every visibility whose footprint touches the core (copies
// included), so every grid cell is accumulated by exactly one workgroup and
// written to HBM once, coalesced, with no global atomics and no separate zero
// fill.  A group of LPV lanes handles one visibility: lane j owns footprint
// column j and loops over the W rows and the W planes.
//
// FP32 path: gfx950 LDS float atomics run at a small fraction of the integer
// rate, so the ring accumulates 64-bit fixed point.  With S = 2^30 / max|z|
// every contribution z phi_u phi_v phi_w (phi <= 1) becomes an exact int32 and
// the int64 sums are exact; the store converts back with 1/S.
// FP64 path: the ring holds doubles updated with LDS float atomics.
constexpr int kTileThreads = 1024;   // 16 waves share one tile's LDS ring

// true for an infinite or NaN float (all exponent bits set); a bit test, so that no
// floating-point contraction or fast-math assumption can change it
__device__ __forceinline__ bool not_finite(float x) { return (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u; }

// Fixed-point scale of the FP32 spread from am >= max |z| of the values spread:
// contributions are z * phi * fscale with |.| <= S, and the stored sums are
// multiplied by finv.  am = 0 means every value is zero (exact zero grid).  An
// am that is not finite (a NaN or infinite value, weight or product) or outside
// [2^-96, 2^120] (where S / am or am / S would leave the FP32 range) turns every
// output cell into NaN (fscale = 0, finv = NaN), so such input is never gridded
// silently.
__device__ __forceinline__ void fixed_point_scale(float am, float S, float &fscale, float &finv) {
    if (am == 0.f) {
        fscale = 1.f;
        finv = 1.f;
    } else if (am >= 0x1p-96f && am <= 0x1p+120f) {
        fscale = S / am;
        finv = am / S;
    } else {
        fscale = 0.f;
        finv = __builtin_nanf("");
    }
}

template <typename R> struct SpreadAcc { using T = R; };
template <> struct SpreadAcc<float> { using T = unsigned long long; };

template <typename R, int W, int LPV, bool FLAT, int VMODE>
__global__ __launch_bounds__(kTileThreads) void spread_kernel(SpreadLaunch a) {
    using A = typename SpreadAcc<R>::T;
    constexpr bool FIX = std::is_same<R, float>::value;
    constexpr int WW = FLAT ? 1 : W;
    constexpr int NT = kTileThreads;
    constexpr int NGRP = NT / LPV;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = a.g.T, TT = T * T;
    A *sre = reinterpret_cast<A *>(smem_raw);
    A *sim = sre + WW * TT;
    const GridWork wk = a.work[blockIdx.x];
    const BandDev bd = a.bands[wk.band];
    const int ntiles = a.g.ntx * a.g.nty;
    const int tu = wk.tile / a.g.nty, tv = wk.tile - tu * a.g.nty;
    const int bb = wk.band - a.band0;
    const Rec<R> *recs = reinterpret_cast<const Rec<R> *>(a.recs);
    const R *omega = reinterpret_cast<const R *>(a.omega);
    const cplx<R> *vis = reinterpret_cast<const cplx<R> *>(a.vis);
    cplx<R> *planes = reinterpret_cast<cplx<R> *>(a.planes);
    // fixed-point scale (FP32 path)
    R fscale = R(1), finv = R(1);
    if constexpr (FIX) fixed_point_scale(*a.absmax, 1073741824.0f, fscale, finv);   // 2^30 / max|z|

    for (int k = threadIdx.x; k < 2 * WW * TT; k += NT) sre[k] = A(0);
    __syncthreads();

    const int lane = threadIdx.x % LPV;
    const int grp = threadIdx.x / LPV;
    const R beta = (R)a.g.beta, inv_hw = R(2) / R(W), hw = R(0.5) * R(W);
    const R w0 = (R)bd.w0, dw = (R)bd.dw, sc = (R)bd.sc;
    const int64_t keybase = ((int64_t)wk.band * ntiles + wk.tile) * a.g.nj0max;
    const int qstart = FLAT ? 0 : max(0, wk.p0 - W + 1);
    const size_t plane_sz = (size_t)a.g.gx * a.g.gy;

    for (int q = qstart; q < wk.p1; ++q) {
        if (q < bd.nj0) {
            // each lane group takes a contiguous run of the bucket, so the groups
            // working at the same time sit far apart in it (different baselines)
            const int64_t b0 = a.offsets[keybase + q], n = a.offsets[keybase + q + 1] - b0;
            const int64_t per = (n + NGRP - 1) / NGRP;
            const int64_t e_beg = b0 + min(n, grp * per), e_end = b0 + min(n, (grp + 1) * per);
            for (int64_t e = e_beg; e < e_end; ++e) {
                const Rec<R> rec = recs[e];
                const uint32_t vid = rec.idx & ~kHomeBit;
                cplx<R> z;
                if (VMODE == 0) {
                    const R om = omega[e];
                    const cplx<R> v = vis[vid];
                    z = v * cis_cycles<R>((w0 + rec.fw * dw) * sc) * om;
                } else if (VMODE == 1) {
                    z = cplx<R>{omega[e], R(0)};
                } else {
                    z = vis[a.home_pos[e]];
                }
                const int i0 = (int)dev_floor(rec.fu - hw) + 1;
                const int j0 = (int)dev_floor(rec.fv - hw) + 1;
                R pu = R(0), pv = R(0), pw = R(1);
                if (lane < W) {
                    pu = es_kernel<R>(R(i0 + lane) - rec.fu, beta, inv_hw);
                    pv = es_kernel<R>(R(j0 + lane) - rec.fv, beta, inv_hw);
                    if (!FLAT) pw = es_kernel<R>(R(q + lane) - rec.fw, beta, inv_hw);
                }
                R wu[W];
#pragma unroll
                for (int i = 0; i < W; ++i) wu[i] = __shfl(pu, i, LPV);
                R ww[WW];
                if (FLAT) {
                    ww[0] = R(1);
                } else {
#pragma unroll
                    for (int k = 0; k < WW; ++k) ww[k] = __shfl(pw, k, LPV);
                }
                const int c = j0 + lane;
                const bool cok = (lane < W) && (c >= 0) && (c < T);
                const cplx<R> zv = z * (pv * fscale);
#pragma unroll
                for (int k = 0; k < WW; ++k) {
                    const int p = q + k;
                    if (!FLAT && (p < wk.p0 || p >= wk.p1)) continue;
                    const int slot = FLAT ? 0 : p % W;
                    A *re = sre + slot * TT + c;
                    A *im = sim + slot * TT + c;
                    const cplx<R> zk = zv * ww[k];
#pragma unroll
                    for (int i = 0; i < W; ++i) {
                        const int row = i0 + i;
                        if (cok && row >= 0 && row < T) {
                            if constexpr (FIX) {
                                const long long qr = (long long)__float2int_rn(zk.re * wu[i]);
                                const long long qi = (long long)__float2int_rn(zk.im * wu[i]);
                                atomicAdd(re + row * T, (unsigned long long)qr);
                                atomicAdd(im + row * T, (unsigned long long)qi);
                            } else {
                                atomicAdd(re + row * T, zk.re * wu[i]);
                                atomicAdd(im + row * T, zk.im * wu[i]);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        const int slot = FLAT ? 0 : q % W;
        if (FLAT || q >= wk.p0) {
            cplx<R> *dst = planes + ((size_t)bb * a.g.nwmax + q) * plane_sz + (size_t)tu * T * a.g.gy + (size_t)tv * T;
            for (int k = threadIdx.x; k < TT; k += NT) {
                const int row = k / T, col = k - row * T;
                cplx<R> v;
                if constexpr (FIX) {
                    v = cplx<R>{(R)((double)(long long)sre[slot * TT + k] * (double)finv),
                                (R)((double)(long long)sim[slot * TT + k] * (double)finv)};
                } else {
                    v = cplx<R>{sre[slot * TT + k], sim[slot * TT + k]};
                }
                dst[(size_t)row * a.g.gy + col] = v;
            }
        }
        for (int k = threadIdx.x; k < TT; k += NT) {
            sre[slot * TT + k] = A(0);
            sim[slot * TT + k] = A(0);
        }
        __syncthreads();
    }
}

// FP32 spread over sorted buckets: one wave per visibility, register
// accumulation across runs of visibilities that share a footprint.
//
// Buckets are sorted by footprint base cell (i0, j0), so consecutive entries
// often cover the same W x W x W block.  Each wave takes a contiguous part of a
// bucket; lane (j, k) owns footprint column j and plane q + k and keeps the W
// row sums of its column in registers; when the base cell changes (or after
// kRunMax visibilities) the wave adds its block to the LDS ring (64-bit fixed
// point, ds_add_u64).  Values are pre-scaled by S = 2^26 / max|z|, so a partial
// sum of at most kRunMax = 31 contributions is below 2^31 in magnitude and
// converts to int32 with one truncation (zero-mean for values of either sign,
// relative size 2^-26 for one-signed sums).  The per-visibility quantities
// (1-D ES weights, z) are computed for 8 visibilities at once, one visibility
// per 8-lane group, then broadcast with readlane / shuffles.  The wave index,
// the bucket range and the run state are wave-uniform (scalar registers).
// FLAT (PSF gridder, one plane): lane (j, i) owns cell (i, j) of the footprint.
constexpr int kRunMax = 31;
constexpr float kRunScale = 67108864.0f;   // 2^26
// LDS stride of one plane slot, in 64-bit words.  A flush touches 7 columns of
// 7 plane slots at once; padding each slot by 2 words spreads those 49
// addresses over the 16 two-bank pairs (at most 4 per pair instead of 7).
__host__ __device__ constexpr int run_slot_stride(int T, bool flat) { return flat ? T * T : T * T + 2; }

__device__ __forceinline__ unsigned long long f2fix(float x) {
    // |x| < 2^31: truncate to int32, sign-extend
    return (unsigned long long)(long long)(int)x;
}
__device__ __forceinline__ float rdlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int rdlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// ES kernel with the hardware square root and base-2 exponential (about one
// ulp each); beta2 = beta * log2(e).
__device__ __forceinline__ float es_kernel_fast(float z, float beta2, float inv_hw) {
    const float t = z * inv_hw;
    const float a = 1.f - t * t;
    return a > 0.f ? __builtin_amdgcn_exp2f(beta2 * (__builtin_amdgcn_sqrtf(a) - 1.f)) : 0.f;
}

template <int W, bool FLAT, int VMODE>
__global__ __launch_bounds__(kTileThreads) void spread_run_kernel(SpreadLaunch a) {
    using R = float;
    using A = unsigned long long;
    constexpr int WW = FLAT ? 1 : W;
    constexpr int NACC = FLAT ? 1 : W;
    constexpr int NWAVE = kTileThreads / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = a.g.T, TT = T * T, TS = run_slot_stride(T, FLAT);
    A *sre = reinterpret_cast<A *>(smem_raw);
    A *sim = sre + WW * TS;
    const GridWork wk = a.work[blockIdx.x];
    const BandDev bd = a.bands[wk.band];
    const int ntiles = a.g.ntx * a.g.nty;
    const int tu = wk.tile / a.g.nty, tv = wk.tile - tu * a.g.nty;
    const int bb = wk.band - a.band0;
    const Rec<R> *recs = reinterpret_cast<const Rec<R> *>(a.recs);
    const R *omega = reinterpret_cast<const R *>(a.omega);
    const cplx<R> *vis = reinterpret_cast<const cplx<R> *>(a.vis);
    cplx<R> *planes = reinterpret_cast<cplx<R> *>(a.planes);
    R fscale = R(1), finv = R(1);
    fixed_point_scale(*a.absmax, kRunScale, fscale, finv);
    for (int k = threadIdx.x; k < 2 * WW * TS; k += kTileThreads) sre[k] = A(0);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lj = lane & 7, ls = lane >> 3;         // column j; plane offset k (or row i when FLAT)
    const bool lact = (lj < W) && (ls < W);
    const R beta2 = (R)(a.g.beta * 1.4426950408889634), inv_hw = R(2) / R(W), hw = R(0.5) * R(W);
    const R w0 = (R)bd.w0, dw = (R)bd.dw, sc = (R)bd.sc;
    const int64_t keybase = ((int64_t)wk.band * ntiles + wk.tile) * a.g.nj0max;
    const int qstart = FLAT ? 0 : max(0, wk.p0 - W + 1);
    const size_t plane_sz = (size_t)a.g.gx * a.g.gy;

    for (int q = qstart; q < wk.p1; ++q) {
        if (q < bd.nj0) {
            const int64_t b0 = a.offsets[keybase + q], n = a.offsets[keybase + q + 1] - b0;
            const int64_t per = (n + NWAVE - 1) / NWAVE;
            const int64_t e_beg = b0 + min(n, wv * per), e_end = b0 + min(n, (wv + 1) * per);
            // this lane's LDS word for footprint cell (row 0, column 0) of a base at (0, 0)
            bool lane_ok;
            int lane_off;
            if (FLAT) {
                lane_ok = lact;
                lane_off = ls * T + lj;
            } else {
                const int p = q + ls;
                lane_ok = lact && p >= wk.p0 && p < wk.p1;
                lane_off = (p % W) * TS + lj;
            }
            R acc_re[NACC], acc_im[NACC];
#pragma unroll
            for (int i = 0; i < NACC; ++i) acc_re[i] = acc_im[i] = R(0);
            int cur = -1, run = 0;
            auto flush = [&](int base) {
                const int i0 = (base >> 16) - 64, j0 = (base & 0xffff) - 64;
                const int c = j0 + lj;
                if (!lane_ok || c < 0 || c >= T) return;
                const int idx0 = lane_off + i0 * T + j0;
                if (FLAT) {
                    const int row = i0 + ls;
                    if (row < 0 || row >= T) return;
                    atomicAdd(sre + idx0, f2fix(acc_re[0]));
                    atomicAdd(sim + idx0, f2fix(acc_im[0]));
                } else {
                    const int ilo = max(0, -i0), ihi = min(W, T - i0);
                    if (ilo == 0 && ihi == W) {
#pragma unroll
                        for (int i = 0; i < W; ++i) {
                            atomicAdd(sre + idx0 + i * T, f2fix(acc_re[i]));
                            atomicAdd(sim + idx0 + i * T, f2fix(acc_im[i]));
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < W; ++i) {
                            if (i >= ilo && i < ihi) {
                                atomicAdd(sre + idx0 + i * T, f2fix(acc_re[i]));
                                atomicAdd(sim + idx0 + i * T, f2fix(acc_im[i]));
                            }
                        }
                    }
                }
            };
            // software pipeline: the record of the next batch and the value it
            // gathers are loaded while the current batch is being accumulated
            auto load_rec = [&](int64_t eb) {
                Rec<R> r{R(0), R(0), R(0), 0u};
                if (eb < e_end) r = recs[eb];
                return r;
            };
            auto load_val = [&](int64_t eb, const Rec<R> &r) {
                cplx<R> v{R(0), R(0)};
                if (eb < e_end) {
                    if (VMODE == 0) {
                        v = vis[r.idx & ~kHomeBit] * (omega[eb] * fscale);
                    } else if (VMODE == 1) {
                        v = cplx<R>{omega[eb] * fscale, R(0)};
                    } else {
                        v = vis[a.home_pos[eb]] * fscale;
                    }
                }
                return v;
            };
            Rec<R> rec_c = load_rec(e_beg + ls);
            cplx<R> val_c = load_val(e_beg + ls, rec_c);
            Rec<R> rec_n = load_rec(e_beg + 8 + ls);
            for (int64_t e = e_beg; e < e_end; e += 8) {
                const int nb = (int)min((int64_t)8, e_end - e);
                // prefetch: value of the next batch, record of the one after
                const cplx<R> val_n = load_val(e + 8 + ls, rec_n);
                const Rec<R> rec_nn = load_rec(e + 16 + ls);
                // batched prologue: group ls handles visibility e + ls, lane lj its 1-D weights
                R pu = R(0), pv = R(0), pw = R(1), zr = R(0), zi = R(0);
                int base = 0;
                if (ls < nb) {
                    const int i0 = (int)dev_floor(rec_c.fu - hw) + 1;
                    const int j0 = (int)dev_floor(rec_c.fv - hw) + 1;
                    base = ((i0 + 64) << 16) | (j0 + 64);
                    if (lj < W) {
                        pu = es_kernel_fast(R(i0 + lj) - rec_c.fu, beta2, inv_hw);
                        pv = es_kernel_fast(R(j0 + lj) - rec_c.fv, beta2, inv_hw);
                        if (!FLAT) pw = es_kernel_fast(R(q + lj) - rec_c.fw, beta2, inv_hw);
                    }
                    cplx<R> z = val_c;
                    if (VMODE == 0) z = z * cis_cycles<R>((w0 + rec_c.fw * dw) * sc);
                    zr = z.re;
                    zi = z.im;
                }
                // all shuffles of the batch first (one LDS round trip), then accumulate
                R wgt[8];
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    wgt[t] = __shfl(pv, t * 8 + lj) * (FLAT ? __shfl(pu, t * 8 + ls) : __shfl(pw, t * 8 + ls));
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (t < nb) {
                        const int src = t * 8;
                        const int bt = rdlane(base, src);
                        if (bt != cur || run == kRunMax) {
                            if (cur >= 0) flush(cur);
#pragma unroll
                            for (int i = 0; i < NACC; ++i) acc_re[i] = acc_im[i] = R(0);
                            cur = bt;
                            run = 0;
                        }
                        ++run;
                        const R cr = rdlane(zr, src) * wgt[t], ci = rdlane(zi, src) * wgt[t];
                        if (FLAT) {
                            acc_re[0] += cr;
                            acc_im[0] += ci;
                        } else {
#pragma unroll
                            for (int i = 0; i < W; ++i) {
                                const R u = rdlane(pu, src + i);
                                acc_re[i] += cr * u;
                                acc_im[i] += ci * u;
                            }
                        }
                    }
                }
                rec_c = rec_n;
                val_c = val_n;
                rec_n = rec_nn;
            }
            if (cur >= 0) flush(cur);
        }
        __syncthreads();
        const int slot = FLAT ? 0 : q % W;
        if (FLAT || q >= wk.p0) {
            cplx<R> *dst = planes + ((size_t)bb * a.g.nwmax + q) * plane_sz + (size_t)tu * T * a.g.gy + (size_t)tv * T;
            for (int k = threadIdx.x; k < TT; k += kTileThreads) {
                const int row = k / T, col = k - row * T;
                dst[(size_t)row * a.g.gy + col] =
                    cplx<R>{(R)((double)(long long)sre[slot * TS + k] * (double)finv),
                            (R)((double)(long long)sim[slot * TS + k] * (double)finv)};
            }
        }
        for (int k = threadIdx.x; k < TT; k += kTileThreads) {
            sre[slot * TS + k] = A(0);
            sim[slot * TS + k] = A(0);
        }
        __syncthreads();
    }
}

// FP32 w-stacked spread on the matrix cores.
//
// For visibilities whose footprints lie in one window of 8 rows, 16 columns
// and the W planes q .. q + W - 1 of a bucket, the gridded block is a sum of
// rank-one terms, G[(k, i), j] = sum_v (P_v[k] U_v[i]) (V_v[j] z_v): a matrix
// product over the visibility index.  v_mfma_f32_16x16x4f32 takes 4
// visibilities per instruction; the M dimension holds two planes x 8 rows per
// 16-row tile (ceil(W / 2) tiles), N the 16 columns, and Re z and Im z are two
// products.  The accumulators of a window stay in registers until the window
// changes (buckets are sorted by window: base rows in blocks of rb = 9 - W,
// base columns in blocks of cb = 17 - W) or kMfmaRunMax visibilities have been
// added; they then go to the LDS plane ring as 64-bit fixed point (ds_add_u64).
//
// Operand layout (one wave, lane l = 16 s + r): A[16 t + r][s] and B[s][r] in
// lane l, result D[16 t + 4 s + v][r] in register v of tile t.  The 16 lanes of
// slot s evaluate the 1-D ES weights of visibility s of the group relative to
// its window: lanes r < 8 the row weight U[r], lanes r >= 8 the plane weight
// P[r - 8], all 16 the column weight V[r]; DPP within the 16-lane row gives
// every lane U[r mod 8] and the plane weights of the tiles.  Slots outside the
// window of an MFMA round get a zero B row.
constexpr int kMfmaRunMax = 124;                // visibilities per flush: 124 * 2^24 < 2^31
constexpr float kMfmaScale = 16777216.0f;       // 2^24
constexpr int kMfmaThreads = 1024;              // 16 waves (at most 128 registers per lane)
template <int W> struct MfmaWin {
    static constexpr int R = 8;                 // window rows
    static constexpr int RB = R - W + 1;        // base rows per window
    static constexpr int CB = 16 - W + 1;       // base columns per window
    static constexpr int NT = (W + 1) / 2;      // 16-row tiles: two planes each
};
void mfma_window(int W, int *rb, int *cb) {
    *rb = 8 - W + 1;
    *cb = 16 - W + 1;
}
typedef float mfma_v4f __attribute__((ext_vector_type(4)));

// DPP within 16-lane rows, bank masks selecting half-rows (banks 0-1 = lanes
// 0-7, banks 2-3 = lanes 8-15); every lane of the row must be active.
// Lanes 8-15 of each 16-lane row take the value of lane r - 8 (row_ror 8 into
// banks 2-3), lanes 0-7 keep their own
__device__ __forceinline__ float row_lo_to_hi(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x128, 0xf, 0xc, false));
}
// lanes 0-7 of each row take lane A of the row, lanes 8-15 lane B
template <int A, int B> __device__ __forceinline__ float row_half_bcast(float v) {
    const int lo = __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + A, 0xf, 0x3, false);
    return __int_as_float(__builtin_amdgcn_update_dpp(lo, __float_as_int(v), 0x150 + B, 0xf, 0xc, false));
}

// a 64-bit value that is the same in every lane, moved to scalar registers
__device__ __forceinline__ int64_t rfl64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// TC: the tile side as a compile-time constant (LDS offsets become immediates), or
// 0 to take it from the launch arguments
template <int W, int VMODE, int TC>
__global__ __launch_bounds__(kMfmaThreads) void spread_mfma_kernel(SpreadLaunch a) {
    using R_ = float;
    using A = unsigned long long;
    constexpr int RB = MfmaWin<W>::RB, CB = MfmaWin<W>::CB, NT = MfmaWin<W>::NT;
    constexpr int NWAVE = kMfmaThreads / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = TC ? TC : a.g.T, TT = T * T, TS = run_slot_stride(T, false);
    A *sre = reinterpret_cast<A *>(smem_raw);
    A *sim = sre + W * TS;
    const GridWork wk = a.work[blockIdx.x];
    const BandDev bd = a.bands[wk.band];
    const int ntiles = a.g.ntx * a.g.nty;
    const int tu = wk.tile / a.g.nty, tv = wk.tile - tu * a.g.nty;
    const int bb = wk.band - a.band0;
    const Rec<R_> *recs = reinterpret_cast<const Rec<R_> *>(a.recs);
    const R_ *omega = reinterpret_cast<const R_ *>(a.omega);
    const cplx<R_> *phase = reinterpret_cast<const cplx<R_> *>(a.phase);
    const cplx<R_> *vis = reinterpret_cast<const cplx<R_> *>(a.vis);
    cplx<R_> *planes = reinterpret_cast<cplx<R_> *>(a.planes);
    R_ fscale = R_(1), finv = R_(1);
    fixed_point_scale(*a.absmax, kMfmaScale, fscale, finv);
    const int64_t keybase = ((int64_t)wk.band * ntiles + wk.tile) * a.g.nj0max;
    const int qstart = max(0, wk.p0 - W + 1);
    const int qlast = min(wk.p1, bd.nj0);        // base planes qstart .. qlast - 1 can hold entries
    // bucket offsets of those base planes: entries of base plane q are
    // soff[q - qstart] .. soff[q - qstart + 1] - 1
    int64_t *soff = reinterpret_cast<int64_t *>(sim + W * TS);
    for (int k = threadIdx.x; k < 2 * W * TS; k += kMfmaThreads) sre[k] = A(0);
    for (int k = threadIdx.x; k <= qlast - qstart; k += kMfmaThreads) soff[k] = a.offsets[keybase + qstart + k];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sg = lane >> 4, r = lane & 15;    // K slot (visibility of a group of 4); row / column
    const R_ beta2 = (R_)(a.g.beta * 1.4426950408889634), inv_hw = R_(2) / R_(W), hw = R_(0.5) * R_(W);
    const size_t plane_sz = (size_t)a.g.gx * a.g.gy;
    auto soff_at = [&](int k) { return rfl64(soff[k]); };   // same address in every lane

    // The entries of a wave form one stream of batches of up to 64: its share of
    // base plane q (1/16 of the bucket), then of the next base plane in which it
    // has a share.  A batch is (q, e, end): entries e .. min(e + 64, end) - 1.
    // Loads run two batches ahead across plane boundaries, so the records and
    // visibilities of the next plane are in flight during this plane's barriers
    // and write-out.
    constexpr int kDone = INT_MAX;
    auto next_batch = [&](int &bq, int64_t &be, int64_t &bend) {
        if (bq == kDone) return;
        be += 64;
        if (be < bend) return;
        for (++bq; bq < qlast; ++bq) {
            const int64_t b0 = soff_at(bq - qstart), n = soff_at(bq - qstart + 1) - b0;
            const int64_t per = (n + NWAVE - 1) / NWAVE;
            be = b0 + min(n, wv * per);
            bend = b0 + min(n, (wv + 1) * per);
            if (be < bend) return;
        }
        bq = kDone;
        be = bend = 0;
    };
    // Loads of lanes past a batch's end read its last entry instead (or entry 0 when
    // the stream is done; the work item has entries): no branch joins a loaded value
    // before its use, which would wait for every load in flight.  Those lanes' slots
    // never reach the matrix products.
    auto clampi = [](int64_t ei, int64_t bend) { return ei < bend ? ei : (bend > 0 ? bend - 1 : (int64_t)0); };
    auto load_rec = [&](int64_t ei, int64_t bend) { return recs[clampi(ei, bend)]; };
    // the value's loads (VMODE 2: through the entry's home position, loaded with its record)
    struct RawVal {
        cplx<R_> z, ph;
        R_ om;
    };
    auto load_val = [&](int64_t ei, int64_t bend, const Rec<R_> &rr, uint32_t hp) {
        const int64_t ec = clampi(ei, bend);
        RawVal raw{{R_(0), R_(0)}, {R_(1), R_(0)}, R_(1)};
        if (VMODE == 0) {
            raw.z = vis[rr.idx & ~kHomeBit];
            raw.ph = phase[ec];
            raw.om = omega[ec];
        } else if (VMODE == 1) {
            raw.om = omega[ec];
        } else {
            raw.z = vis[hp];
        }
        return raw;
    };
    auto make_val = [&](const RawVal &raw) {
        if (VMODE == 0) return raw.z * raw.ph * (raw.om * fscale);
        if (VMODE == 1) return cplx<R_>{raw.om * fscale, R_(0)};
        return raw.z * fscale;
    };
    auto load_hp = [&](int64_t ei, int64_t bend) { return VMODE == 2 ? a.home_pos[clampi(ei, bend)] : 0u; };
    // batch a: records and values loaded; batch b: records (and home positions) loaded
    int qa = qstart - 1, qb;
    int64_t ea = 0, enda = 0, eb, endb;
    next_batch(qa, ea, enda);
    qb = qa;
    eb = ea;
    endb = enda;
    next_batch(qb, eb, endb);
    Rec<R_> rec_c = load_rec(ea + lane, enda);
    RawVal val_c = load_val(ea + lane, enda, rec_c, load_hp(ea + lane, enda));
    Rec<R_> rec_n = load_rec(eb + lane, endb);
    uint32_t hp_n = load_hp(eb + lane, endb);
    unsigned live = 0;    // bit k: base plane q - k has entries in this bucket (planes q - W + 1 .. q)

    for (int q = qstart; q < wk.p1; ++q) {
        const bool has = q < qlast && soff_at(q - qstart + 1) != soff_at(q - qstart);   // block-uniform
        if (qa == q) {
            mfma_v4f cre[NT], cim[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) cre[t] = cim[t] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
            constexpr int kNoRun = INT_MIN;
            int cur = kNoRun, run = 0;
            // LDS word of accumulator (t, v) for a window at the tile origin:
            // plane 2 t + (s >= 2) of the tile, row 4 (s mod 2) + v, column r;
            // koff[t] = -1 when that plane is not stored by this work item
            int koff[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int k = 2 * t + (sg >> 1), p = q + k;
                koff[t] = (k < W && p >= wk.p0 && p < wk.p1) ? (p % W) * TS : -1;
            }
            const int ioff = (4 * (sg & 1)) * T + r;
            // add the accumulators of window `key` to the plane ring and clear them
            auto flush = [&](int key) {
                const int I = ((key >> 8) - 64) * RB - (W - 1), J = ((key & 0xff) - 64) * CB - (W - 1);
                const int base = I * T + J + ioff;
                const bool colok = J + r >= 0 && J + r < T;
                const bool rows_in = I >= 0 && I + 8 <= T;    // wave-uniform
                if (rows_in) {    // one lane mask per tile, no per-row tests
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if (colok && koff[t] >= 0) {
                            const int idx = koff[t] + base;
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                atomicAdd(sre + idx + v * T, f2fix(cre[t][v]));
                                atomicAdd(sim + idx + v * T, f2fix(cim[t][v]));
                            }
                        }
                        cre[t] = cim[t] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
                    }
                    return;
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = I + 4 * (sg & 1) + v;
                        if (colok && koff[t] >= 0 && row >= 0 && row < T) {
                            const int idx = koff[t] + base + v * T;
                            atomicAdd(sre + idx, f2fix(cre[t][v]));
                            atomicAdd(sim + idx, f2fix(cim[t][v]));
                        }
                    }
                    cre[t] = cim[t] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
                }
            };
            // Lane l of a batch holds entry e + l (records coalesced, visibility
            // gathers issued together); a batch is processed in 16 groups of 4.  The
            // owner lane of an entry derives its window and offsets once; each 16-lane
            // slot fetches them with ds_bpermute.
            auto bperm_f = [](int addr, R_ x) {
                return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
            };
            while (qa == q) {
                int qc = qb;
                int64_t ec = eb, endc = endb;
                next_batch(qc, ec, endc);
                const RawVal val_n = load_val(eb + lane, endb, rec_n, hp_n);
                const Rec<R_> rec_nn = load_rec(ec + lane, endc);
                const uint32_t hp_nn = load_hp(ec + lane, endc);
                const cplx<R_> zc = make_val(val_c);
                const int nbatch = (int)min((int64_t)64, enda - ea);
                // owner lane: window of its entry and the offsets of the window origin
                int okey;
                R_ odu, odv, odq;
                {
                    const int i0 = (int)dev_floor(rec_c.fu - hw) + 1;
                    const int j0 = (int)dev_floor(rec_c.fv - hw) + 1;
                    const int wa = floordiv(i0 + W - 1, RB), wb = floordiv(j0 + W - 1, CB);
                    okey = ((wa + 64) << 8) | (wb + 64);
                    odu = R_(wa * RB - (W - 1)) - rec_c.fu;     // row 0 of the window minus fu
                    odv = R_(wb * CB - (W - 1)) - rec_c.fv;
                    odq = R_(q) - rec_c.fw;
                }
                // operands of group 0 of the batch; each group fetches those of the next
                // one before its matrix products, so the crossbar latency overlaps them
                const int own0 = sg * 4;                // byte address of the owner lane
                R_ du = bperm_f(own0, odu), dv = bperm_f(own0, odv), dq = bperm_f(own0, odq);
                R_ zr = bperm_f(own0, zc.re), zi = bperm_f(own0, zc.im);
                int key = __builtin_amdgcn_ds_bpermute(own0, okey);
#pragma unroll 1
                for (int g4 = 0; g4 < nbatch; g4 += 4) {
                    const int nb = min(4, nbatch - g4);
                    const bool hi = r >= 8;               // rows 8..15 of a tile: its second plane
                    // plane weights k = r - 8 >= W fall outside the support (zero) and
                    // their planes are never flushed
                    // the VALU work of a group (weights, operands) and the flushes run at a
                    // raised wave priority, the matrix products at the base one: waves that
                    // compute win the issue arbitration while another wave's products keep
                    // the matrix core busy (6.35 -> 6.01 ms)
                    __builtin_amdgcn_s_setprio(1);
                    const R_ E = es_kernel_fast(hi ? dq + R_(r - 8) : du + R_(r), beta2, inv_hw);
                    const R_ V = es_kernel_fast(dv + R_(r), beta2, inv_hw);
                    const R_ U = row_lo_to_hi(E);         // U[r mod 8]
                    R_ At[NT];                            // U x plane weight (2t, 2t + 1 for rows 8-15)
                    At[0] = U * row_half_bcast<8, 9>(E);
                    if constexpr (NT > 1) At[1] = U * row_half_bcast<10, 11>(E);
                    if constexpr (NT > 2) At[2] = U * row_half_bcast<12, 13>(E);
                    if constexpr (NT > 3) At[3] = U * row_half_bcast<14, 15>(E);
                    const R_ Bre = V * zr, Bim = V * zi;
                    // windows present in this group (wave-uniform); usually one, the
                    // current one: every lane holds the window of its slot
                    const int key0 = rdlane(key, 0);
                    const bool one = nb == 4 && key0 == cur && run + 4 <= kMfmaRunMax &&
                                     __builtin_amdgcn_ballot_w64(key == key0) == ~0ull;
                    const int keyv = key;
                    {
                        // next group (after the last group of the batch: unused)
                        const int own = ((g4 + 4 + sg) & 63) * 4;
                        du = bperm_f(own, odu);
                        dv = bperm_f(own, odv);
                        dq = bperm_f(own, odq);
                        zr = bperm_f(own, zc.re);
                        zi = bperm_f(own, zc.im);
                        key = __builtin_amdgcn_ds_bpermute(own, okey);
                    }
                    __builtin_amdgcn_s_setprio(0);
                    unsigned rem = (1u << nb) - 1u;
                    while (rem) {
                        int w = key0;
                        unsigned sel = 0xfu;    // four entries of the current window
                        if (!one) {
                            int keys[4];
#pragma unroll
                            for (int g = 0; g < 4; ++g) keys[g] = rdlane(keyv, 16 * g);
                            const int f = __builtin_ctz(rem);
#pragma unroll
                            for (int g = 1; g < 4; ++g)
                                if (f == g) w = keys[g];
                            sel = 0;
#pragma unroll
                            for (int g = 0; g < 4; ++g)
                                if (((rem >> g) & 1u) && keys[g] == w) sel |= 1u << g;
                        }
                        const int cnt = __builtin_popcount(sel);
                        if (w != cur || run + cnt > kMfmaRunMax) {
                            __builtin_amdgcn_s_setprio(1);
                            if (cur != kNoRun) flush(cur);
                            __builtin_amdgcn_s_setprio(0);
                            cur = w;
                            run = 0;
                        }
                        run += cnt;
                        // slots of other windows contribute nothing: zero their B rows
                        const bool mine = (sel >> sg) & 1u;
                        const R_ bre = mine ? Bre : R_(0), bim = mine ? Bim : R_(0);
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            cre[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(At[t], bre, cre[t], 0, 0, 0);
                            cim[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(At[t], bim, cim[t], 0, 0, 0);
                        }
                        rem &= ~sel;
                    }
                }
                rec_c = rec_n;
                val_c = val_n;
                rec_n = rec_nn;
                hp_n = hp_nn;
                qa = qb;
                ea = eb;
                enda = endb;
                qb = qc;
                eb = ec;
                endb = endc;
            }
            if (cur != kNoRun) flush(cur);
        }
        // planes without any entry of base planes q - W + 1 .. q are zero: not
        // written (the transforms read only occupied tiles), and their LDS slot
        // stays zero; a plane without atomics needs no barrier before its write-out
        if (has) __syncthreads();
        live = ((live << 1) | (has ? 1u : 0u)) & ((1u << W) - 1u);
        if (!live) continue;
        const int slot = q % W;
        if (q >= wk.p0) {
            cplx<R_> *dst = planes + ((size_t)bb * a.g.nwmax + q) * plane_sz + (size_t)tu * T * a.g.gy + (size_t)tv * T;
            for (int k = threadIdx.x; k < TT; k += kMfmaThreads) {
                const int row = k / T, col = k - row * T;
                dst[(size_t)row * a.g.gy + col] =
                    cplx<R_>{(R_)((double)(long long)sre[slot * TS + k] * (double)finv),
                             (R_)((double)(long long)sim[slot * TS + k] * (double)finv)};
            }
        }
        for (int k = threadIdx.x; k < TT; k += kMfmaThreads) {
            sre[slot * TS + k] = A(0);
            sim[slot * TS + k] = A(0);
        }
        __syncthreads();
    }
}

// max |z| over active visibilities (FP32 path): per-block maxima, then one block
__global__ __launch_bounds__(kThreads) void absmax_blocks_kernel(int vmode, const cplx<float> *vis,
                                                                 const float *weight, const uint8_t *flag,
                                                                 int64_t n, float *partials) {
    __shared__ float red[kThreads / 64];
    // per entry |w z| <= w hypot(|Re z|, |Im z|), the hypot formed without squaring
    // in FP32 (max * sqrt(1 + (min / max)^2)); a NaN or infinite weight, value or
    // product makes the bound infinite.  U entries per thread at a time: all their
    // loads (indices clamped, not tested; the flag and value reads fixed per
    // instantiation) before any use, so that they are in flight together.
    float m = 0.f;
    bool bad = false;
    auto run = [&](auto HASF, auto VM) {
        constexpr bool HF = decltype(HASF)::value;
        constexpr int VMODE = decltype(VM)::value;
        constexpr int U = 4;
        const int64_t stride = (int64_t)gridDim.x * kThreads;
        for (int64_t e0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; e0 < n; e0 += U * stride) {
            float w[U];
            uint8_t f[U];
            cplx<float> z[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t e = min(e0 + u * stride, n - 1);
                w[u] = weight[e];
                f[u] = HF ? flag[e] : 0;
                if (VMODE != 1) z[u] = vis[e];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // (past the end: off, not a branch, which would let the compiler sink the loads)
                const bool on = e0 + u * stride < n && w[u] > 0.f && !f[u];
                float v = w[u];
                if (VMODE != 1) {
                    const float ar = fabsf(z[u].re), ai = fabsf(z[u].im);
                    const float hi = fmaxf(ar, ai), lo = fminf(ar, ai);
                    const float t = hi > 0.f ? lo / hi : 0.f;
                    v = hi * sqrtf(1.f + t * t) * (VMODE == 0 ? w[u] : 1.f);
                    if (on) bad = bad || not_finite(z[u].re) || not_finite(z[u].im);
                }
                if (on) {
                    m = fmaxf(m, v);
                    bad = bad || not_finite(v);
                }
            }
        }
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    using V0 = std::integral_constant<int, 0>;
    using V1 = std::integral_constant<int, 1>;
    using V2 = std::integral_constant<int, 2>;
    if (flag) {
        if (vmode == 0) run(T_{}, V0{});
        else if (vmode == 1) run(T_{}, V1{});
        else run(T_{}, V2{});
    } else {
        if (vmode == 0) run(F_{}, V0{});
        else if (vmode == 1) run(F_{}, V1{});
        else run(F_{}, V2{});
    }
    if (bad) m = INFINITY;
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < kThreads / 64; ++k) t = fmaxf(t, red[k]);
        partials[blockIdx.x] = t;
    }
}
__global__ __launch_bounds__(kThreads) void absmax_final_kernel(const float *partials, int n, float *out) {
    __shared__ float red[kThreads / 64];
    float m = 0.f;
    for (int k = threadIdx.x; k < n; k += kThreads) m = fmaxf(m, partials[k]);
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < kThreads / 64; ++k) t = fmaxf(t, red[k]);
        // margin so that rounding in z * phi * S never exceeds 2^31 - 1
        out[0] = t * 1.0001f;
    }
}
__global__ void absmax_clear_kernel(float *out) { out[0] = 0.f; }
hipError_t launch_absmax_clear(float *absmax, hipStream_t s) {
    PFB_LAUNCH_NT(absmax_clear_kernel, 1, 64, 0, s, absmax);
    return hipSuccess;
}
hipError_t launch_absmax(int vmode, const void *vis, const void *weight, const uint8_t *flag, int64_t n,
                         float *partials, float *absmax, hipStream_t s) {
    int64_t nb = (n + kThreads - 1) / kThreads;
    if (nb > kAbsmaxBlocks) nb = kAbsmaxBlocks;
    if (nb < 1) nb = 1;
    PFB_LAUNCH(absmax_blocks_kernel, nb, 0, s, vmode, (const cplx<float> *)vis, (const float *)weight, flag, n,
               partials);
    PFB_LAUNCH(absmax_final_kernel, 1, 0, s, partials, (int)nb, absmax);
    return hipSuccess;
}

template <typename R, int W, int LPV>
static hipError_t spread_w(const SpreadLaunch &a, hipStream_t s) {
    const bool flat = a.g.flat;
    const size_t lds = 2 * (size_t)(flat ? 1 : W) * a.g.T * a.g.T * sizeof(typename SpreadAcc<R>::T);
#define SPREAD_CASE(FL, VM)                                                         \
    if (flat == FL && a.vmode == VM) {                                              \
        PFB_LAUNCH_NT((spread_kernel<R, W, LPV, FL, VM>), a.n_work, kTileThreads, lds, s, a); \
        return hipSuccess;                                                          \
    }
    SPREAD_CASE(false, 0)
    SPREAD_CASE(false, 1)
    SPREAD_CASE(false, 2)
    SPREAD_CASE(true, 0)
    SPREAD_CASE(true, 1)
    SPREAD_CASE(true, 2)
#undef SPREAD_CASE
    return hipErrorInvalidValue;
}

template <int W>
static hipError_t spread_run_w(const SpreadLaunch &a, hipStream_t s) {
    const bool flat = a.g.flat;
    if (!flat && a.phase) {
        // plane ring + bucket offsets of the base planes of one work item
        const size_t lds = 2 * (size_t)W * run_slot_stride(a.g.T, false) * sizeof(unsigned long long) +
                           ((size_t)a.g.nj0max + 1) * sizeof(int64_t);
        if (a.g.T == 32) {   // the default tile
            if (a.vmode == 0) PFB_LAUNCH_NT((spread_mfma_kernel<W, 0, 32>), a.n_work, kMfmaThreads, lds, s, a);
            else if (a.vmode == 1) PFB_LAUNCH_NT((spread_mfma_kernel<W, 1, 32>), a.n_work, kMfmaThreads, lds, s, a);
            else PFB_LAUNCH_NT((spread_mfma_kernel<W, 2, 32>), a.n_work, kMfmaThreads, lds, s, a);
        } else {
            if (a.vmode == 0) PFB_LAUNCH_NT((spread_mfma_kernel<W, 0, 0>), a.n_work, kMfmaThreads, lds, s, a);
            else if (a.vmode == 1) PFB_LAUNCH_NT((spread_mfma_kernel<W, 1, 0>), a.n_work, kMfmaThreads, lds, s, a);
            else PFB_LAUNCH_NT((spread_mfma_kernel<W, 2, 0>), a.n_work, kMfmaThreads, lds, s, a);
        }
        return hipSuccess;
    }
    const size_t lds = 2 * (size_t)(flat ? 1 : W) * run_slot_stride(a.g.T, flat) * sizeof(unsigned long long);
#define SPREAD_RUN_CASE(FL, VM)                                                                 \
    if (flat == FL && a.vmode == VM) {                                                          \
        PFB_LAUNCH_NT((spread_run_kernel<W, FL, VM>), a.n_work, kTileThreads, lds, s, a);       \
        return hipSuccess;                                                                      \
    }
    SPREAD_RUN_CASE(false, 0)
    SPREAD_RUN_CASE(false, 1)
    SPREAD_RUN_CASE(false, 2)
    SPREAD_RUN_CASE(true, 0)
    SPREAD_RUN_CASE(true, 1)
    SPREAD_RUN_CASE(true, 2)
#undef SPREAD_RUN_CASE
    return hipErrorInvalidValue;
}

// cplx<float> after the LDS ring of the FP32 interpolation (reads of zero-weight
// columns), and zero columns after each ring row (row stride T + W + kInterp4ColPad)
constexpr int kInterp4Pad = 8;
constexpr int kInterp4ColPad = 1;

size_t gridder_lds_bytes(bool dbl, int W, int T, bool flat) {
    const size_t ww = flat ? 1 : (size_t)W;
    const size_t spread = dbl ? 2 * ww * T * T * sizeof(double)
                              : 2 * ww * run_slot_stride(T, flat) * sizeof(unsigned long long);
    const size_t interp = (ww * (size_t)(T + W) * (T + W + (dbl ? 0 : kInterp4ColPad)) + (dbl ? 0 : kInterp4Pad)) *
                          (dbl ? sizeof(cplx<double>) : sizeof(cplx<float>));
    return spread > interp ? spread : interp;
}

hipError_t launch_spread(bool dbl, const SpreadLaunch &a, hipStream_t s) {
    if (a.n_work <= 0) return hipSuccess;
    if (dbl)
        return dispatch_int<9, 16>(a.g.W, [&](auto Wc) { return spread_w<double, decltype(Wc)::value, 16>(a, s); });
    return dispatch_int<4, 8>(a.g.W, [&](auto Wc) { return spread_run_w<decltype(Wc)::value>(a, s); });
}

// ---------------------------------------------------------------------------
// degridding: halo subgrid of W w-planes in an LDS ring
// ---------------------------------------------------------------------------
// A work item covers a run of entries of one tile sorted by base plane; it
// keeps the (T+W) x (T+W) halo region of W consecutive w-planes in LDS and
// slides one plane at a time.  Each visibility is computed once, from its home
// tile; lanes of a group own footprint columns and the partial sums are
// reduced across the group with lane shuffles.
// FP64 mode: `interp_kernel` (LPV lanes per visibility, lane shuffles); FP32:
// `interp4_kernel` below.
template <typename R, int W, int LPV, bool FLAT, int OMODE>
__global__ __launch_bounds__(kTileThreads) void interp_kernel(InterpLaunch a) {
    constexpr int WW = FLAT ? 1 : W;
    constexpr int NT = kTileThreads;
    constexpr int NGRP = NT / LPV;
    constexpr int H = (W - 1) / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *ring = reinterpret_cast<cplx<R> *>(smem_raw);
    const int T = a.g.T, S = T + W, SS = S * S;
    const InterpWork wk = a.work[blockIdx.x];
    const BandDev bd = a.bands[wk.band];
    const int ntiles = a.g.ntx * a.g.nty;
    const int tu = wk.tile / a.g.nty, tv = wk.tile - tu * a.g.nty;
    const int bb = wk.band - a.band0;
    const Rec<R> *recs = reinterpret_cast<const Rec<R> *>(a.recs);
    const R *omega = reinterpret_cast<const R *>(a.omega);
    const size_t plane_sz = (size_t)a.g.gx * a.g.gy;
    const cplx<R> *pbase = reinterpret_cast<const cplx<R> *>(a.planes) + (size_t)bb * a.g.nwmax * plane_sz;
    const int gx = a.g.gx, gy = a.g.gy;
    const int ox = tu * T - H, oy = tv * T - H;

    auto load_plane = [&](int p, int slot) {
        const cplx<R> *P = pbase + (size_t)p * plane_sz;
        cplx<R> *dst = ring + slot * SS;
        for (int k = threadIdx.x; k < SS; k += NT) {
            const int aa = k / S, cc = k - aa * S;
            const int gi = wrapi(ox + aa, gx), gj = wrapi(oy + cc, gy);
            dst[k] = P[(size_t)gi * gy + gj];
        }
    };

    for (int k = 0; k < WW; ++k)
        if (wk.q0 + k < (FLAT ? 1 : bd.nw)) load_plane(wk.q0 + k, (wk.q0 + k) % WW);
    __syncthreads();

    const int lane = threadIdx.x % LPV;
    const int grp = threadIdx.x / LPV;
    const R beta = (R)a.g.beta, inv_hw = R(2) / R(W), hw = R(0.5) * R(W);
    const R w0 = (R)bd.w0, dw = (R)bd.dw, sc = (R)bd.sc;
    const int64_t keybase = ((int64_t)wk.band * ntiles + wk.tile) * a.g.nj0max;

    for (int q = wk.q0; q <= wk.q1; ++q) {
        const int64_t lo = max((int64_t)wk.e0, a.hoffsets[keybase + q]);
        const int64_t hi = min((int64_t)wk.e1, a.hoffsets[keybase + q + 1]);
        // group grp takes entries lo + grp, lo + grp + NGRP, ...: the groups of a
        // wave read neighbouring footprints (same window)
        const int64_t n = max(hi - lo, (int64_t)0);
        const int64_t e_end = lo + n;
        for (int64_t h = lo + grp; h < e_end; h += NGRP) {
            const int64_t e = a.hidx[h];        // entry listed under its own tile
            const Rec<R> rec = recs[e];
            const int i0 = (int)dev_floor(rec.fu - hw) + 1;
            const int j0 = (int)dev_floor(rec.fv - hw) + 1;
            R pu = R(0), pv = R(0), pw = R(1);
            if (lane < W) {
                pu = es_kernel<R>(R(i0 + lane) - rec.fu, beta, inv_hw);
                pv = es_kernel<R>(R(j0 + lane) - rec.fv, beta, inv_hw);
                if (!FLAT) pw = es_kernel<R>(R(q + lane) - rec.fw, beta, inv_hw);
            }
            R wu[W];
            R ww[WW];
#pragma unroll
            for (int i = 0; i < W; ++i) wu[i] = __shfl(pu, i, LPV);
            if (FLAT) {
                ww[0] = R(1);
            } else {
#pragma unroll
                for (int k = 0; k < WW; ++k) ww[k] = __shfl(pw, k, LPV);
            }
            cplx<R> acc{R(0), R(0)};
            if (lane < W) {
                const int col = j0 + lane + H;
#pragma unroll
                for (int k = 0; k < WW; ++k) {
                    const cplx<R> *base = ring + ((q + k) % WW) * SS + col;
                    cplx<R> ak{R(0), R(0)};
#pragma unroll
                    for (int i = 0; i < W; ++i) {
                        const cplx<R> g = base[(i0 + i + H) * S];
                        ak.re += wu[i] * g.re;
                        ak.im += wu[i] * g.im;
                    }
                    acc.re += ww[k] * ak.re;
                    acc.im += ww[k] * ak.im;
                }
                acc.re *= pv;
                acc.im *= pv;
            }
#pragma unroll
            for (int off = LPV / 2; off >= 1; off >>= 1) {
                acc.re += __shfl_xor(acc.re, off, LPV);
                acc.im += __shfl_xor(acc.im, off, LPV);
            }
            if (lane == 0) {
                const uint32_t vid = rec.idx & ~kHomeBit;
                if (OMODE != 1) {
                    cplx<R> out = FLAT ? acc : acc * conj(cis_cycles<R>((w0 + rec.fw * dw) * sc));
                    cplx<R> *ov = reinterpret_cast<cplx<R> *>(a.out) + vid;
                    *ov = OMODE == 2 ? *ov + out : out;
                } else {
                    const cplx<R> o = acc * omega[e];
                    reinterpret_cast<cplx<R> *>(a.out)[h] = o;   // home-list order
                }
            }
        }
        __syncthreads();
        if (!FLAT && q < wk.q1 && q + W < bd.nw) {
            load_plane(q + W, q % W);
        }
        __syncthreads();
    }
}

// FP32 interpolation with 4 lanes per visibility (W <= 8): lane q of a quad owns
// footprint columns q and q + 4 (the two 8-byte LDS reads merge into one
// ds_read2_b64; each half reads 32 contiguous bytes per quad, as the 8-lane
// version reads 64), evaluates those two column weights and its share of the row and
// plane weights (indices q and q + 4), which quad_perm DPP broadcasts to the quad;
// a wave interpolates 16 visibilities at a time.  Columns at or beyond W have zero
// weight; their reads stay inside the ring (the next row, or the zeroed pad after
// the last one).
template <int I> __device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), I * 0x55, 0xf, 0xf, false));
}
__device__ __forceinline__ float quad_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4e, 0xf, 0xf, false));
    return v;
}
template <int W, int I = 0> __device__ __forceinline__ void quad_bcast_w(float a, float b, float *out) {
    if constexpr (I < W) {
        out[I] = I < 4 ? quad_bcast<I & 3>(a) : quad_bcast<I & 3>(b);
        quad_bcast_w<W, I + 1>(a, b, out);
    }
}

template <int W, bool FLAT, int OMODE>
__global__ __launch_bounds__(kTileThreads) void interp4_kernel(InterpLaunch a) {
    using R = float;
    static_assert(W <= 8, "two columns per lane, four lanes");
    constexpr int WW = FLAT ? 1 : W;
    constexpr int NT = kTileThreads;
    constexpr int NGRP = NT / 4;
    constexpr int H = (W - 1) / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *ring = reinterpret_cast<cplx<R> *>(smem_raw);
    // ring rows hold the E = T + W halo columns, kInterp4ColPad zero columns after them
    const int T = a.g.T, E = T + W, S = E + kInterp4ColPad, SS = E * S;
    const InterpWork wk = a.work[blockIdx.x];
    const BandDev bd = a.bands[wk.band];
    const int ntiles = a.g.ntx * a.g.nty;
    const int tu = wk.tile / a.g.nty, tv = wk.tile - tu * a.g.nty;
    const int bb = wk.band - a.band0;
    const Rec<R> *recs = reinterpret_cast<const Rec<R> *>(a.recs);
    const R *omega = reinterpret_cast<const R *>(a.omega);
    const size_t plane_sz = (size_t)a.g.gx * a.g.gy;
    const cplx<R> *pbase = reinterpret_cast<const cplx<R> *>(a.planes) + (size_t)bb * a.g.nwmax * plane_sz;
    const int gx = a.g.gx, gy = a.g.gy;
    const int ox = tu * T - H, oy = tv * T - H;

    // value k of the E x E footprint of plane p (row k / E, column k mod E, wrapped)
    auto fetch = [&](int p, int k) {
        const int aa = k / E, cc = k - aa * E;
        return pbase[(size_t)p * plane_sz + (size_t)wrapi(ox + aa, gx) * gy + wrapi(oy + cc, gy)];
    };
    auto put = [&](int p, int k, const cplx<R> &v) {
        const int aa = k / E;
        ring[(p % WW) * SS + aa * S + k - aa * E] = v;
    };
    // the footprints of planes pa .. pb - 1 into their ring slots, eight loads per
    // thread in flight before their LDS writes
    auto load_planes = [&](int pa, int pb) {
        const int per = E * E, total = (pb - pa) * per;
        constexpr int U = 8;
        for (int k0 = threadIdx.x; k0 < total; k0 += U * NT) {
            cplx<R> v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + u * NT, pl = k / per;
                if (k < total) v[u] = fetch(pa + pl, k - pl * per);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + u * NT, pl = k / per;
                if (k < total) put(pa + pl, k - pl * per, v[u]);
            }
        }
    };
    if (threadIdx.x < kInterp4Pad) ring[WW * SS + threadIdx.x] = cplx<R>{R(0), R(0)};
    if constexpr (kInterp4ColPad > 0)
        for (int k = threadIdx.x; k < WW * E * kInterp4ColPad; k += NT) {
            const int r = k / kInterp4ColPad, c = k - r * kInterp4ColPad;
            ring[r * S + E + c] = cplx<R>{R(0), R(0)};
        }
    load_planes(wk.q0, min(wk.q0 + WW, FLAT ? 1 : bd.nw));
    __syncthreads();
    // the plane that replaces plane q in the ring is loaded into registers before
    // q's entries are processed (footprints of up to kPre NT values)
    constexpr int kPre = 2;
    const bool pre_ok = E * E <= kPre * NT;

    const int lq = threadIdx.x & 3;
    const int grp = threadIdx.x >> 2;
    const R inv_hw = R(2) / R(W), hw = R(0.5) * R(W);
    const float beta2 = (float)(a.g.beta * 1.4426950408889634);
    const R w0 = (R)bd.w0, dw = (R)bd.dw, sc = (R)bd.sc;
    const int64_t keybase = ((int64_t)wk.band * ntiles + wk.tile) * a.g.nj0max;

    // OMODE 1: largest |Re| and |Im| of the values written (scale of the FP32 spread
    // that follows); vbad: some value is NaN or infinite
    R vmre = R(0), vmim = R(0);
    bool vbad = false;
    for (int q = wk.q0; q <= wk.q1; ++q) {
        const bool refill = !FLAT && q < wk.q1 && q + W < bd.nw;
        cplx<R> pre[kPre];
        if (refill && pre_ok) {
#pragma unroll
            for (int u = 0; u < kPre; ++u) {
                const int k = threadIdx.x + u * NT;
                if (k < E * E) pre[u] = fetch(q + W, k);
            }
        }
        const int64_t lo = max((int64_t)wk.e0, a.hoffsets[keybase + q]);
        const int64_t hi = min((int64_t)wk.e1, a.hoffsets[keybase + q + 1]);
        const int64_t n = max(hi - lo, (int64_t)0);
        const int64_t e_end = lo + n;
        int64_t h = lo + grp;
        int64_t e_n = 0, e_nn = 0;
        Rec<R> rec_n{R(0), R(0), R(0), 0u};
        // the stored phase of the next entry (degridding with stored phases), loaded with its record
        constexpr bool PH = OMODE != 1 && !FLAT;
        const cplx<R> *phs = reinterpret_cast<const cplx<R> *>(a.phase);
        cplx<R> ph_n{R(1), R(0)};
        R om_n = R(0);   // the weight of the next entry (OMODE 1)
        // the loads of the next two entries run ahead of this one's arithmetic; their
        // indices are clamped to the last entry instead of tested, so that no branch
        // joins a load's value before it is used (that would wait for every load in flight)
        if (h < e_end) {
            e_n = a.hidx[h];
            rec_n = recs[e_n];
            if (PH && a.use_phase) ph_n = phs[e_n];
            if (OMODE == 1) om_n = omega[e_n];
            e_nn = a.hidx[min(h + NGRP, e_end - 1)];
        }
        for (; h < e_end; h += NGRP) {
            const Rec<R> rec = rec_n;
            const cplx<R> ph = ph_n;
            const R om = om_n;
            e_n = e_nn;
            rec_n = recs[e_n];
            if (PH && a.use_phase) ph_n = phs[e_n];
            if (OMODE == 1) om_n = omega[e_n];
            e_nn = a.hidx[min(h + 2 * NGRP, e_end - 1)];
            const int i0 = (int)dev_floor(rec.fu - hw) + 1;
            const int j0 = (int)dev_floor(rec.fv - hw) + 1;
            const R pv0 = es_kernel_fast(R(j0 + lq) - rec.fv, beta2, inv_hw);
            const R pv1 = es_kernel_fast(R(j0 + lq + 4) - rec.fv, beta2, inv_hw);
            const R pua = es_kernel_fast(R(i0 + lq) - rec.fu, beta2, inv_hw);
            const R pub = es_kernel_fast(R(i0 + lq + 4) - rec.fu, beta2, inv_hw);
            R wu[W];
            quad_bcast_w<W>(pua, pub, wu);
            R ww[WW];
            if constexpr (FLAT) {
                ww[0] = R(1);
            } else {
                const R pwa = es_kernel_fast(R(q + lq) - rec.fw, beta2, inv_hw);
                const R pwb = es_kernel_fast(R(q + lq + 4) - rec.fw, beta2, inv_hw);
                quad_bcast_w<WW>(pwa, pwb, ww);
            }
            const int col = j0 + lq + H;
            cplx<R> A0{R(0), R(0)}, A1{R(0), R(0)};
#pragma unroll
            for (int k = 0; k < WW; ++k) {
                const cplx<R> *base = ring + ((q + k) % WW) * SS + col;
                cplx<R> a0{R(0), R(0)}, a1{R(0), R(0)};
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const cplx<R> *row = base + (i0 + i + H) * S;
                    const cplx<R> g0 = row[0], g1 = row[4];
                    a0.re += wu[i] * g0.re;
                    a0.im += wu[i] * g0.im;
                    a1.re += wu[i] * g1.re;
                    a1.im += wu[i] * g1.im;
                }
                A0.re += ww[k] * a0.re;
                A0.im += ww[k] * a0.im;
                A1.re += ww[k] * a1.re;
                A1.im += ww[k] * a1.im;
            }
            cplx<R> acc{pv0 * A0.re + pv1 * A1.re, pv0 * A0.im + pv1 * A1.im};
            acc.re = quad_sum(acc.re);
            acc.im = quad_sum(acc.im);
            if (lq == 0) {
                const uint32_t vid = rec.idx & ~kHomeBit;
                if (OMODE != 1) {
                    cplx<R> out = acc;
                    if (!FLAT) out = out * conj(a.use_phase ? ph : cis_cycles<R>((w0 + rec.fw * dw) * sc));
                    cplx<R> *ov = reinterpret_cast<cplx<R> *>(a.out) + vid;
                    *ov = OMODE == 2 ? *ov + out : out;
                } else {
                    const cplx<R> o = acc * om;
                    reinterpret_cast<cplx<R> *>(a.out)[h] = o;   // home-list order
                    vmre = max(vmre, fabsf(o.re));
                    vmim = max(vmim, fabsf(o.im));
                    vbad = vbad || not_finite(o.re) || not_finite(o.im);
                }
            }
        }
        __syncthreads();
        if (refill) {
            if (pre_ok) {
#pragma unroll
                for (int u = 0; u < kPre; ++u) {
                    const int k = threadIdx.x + u * NT;
                    if (k < E * E) put(q + W, k, pre[u]);
                }
            } else {
                load_planes(q + W, q + W + 1);
            }
        }
        __syncthreads();
    }
    if constexpr (OMODE == 1) {
        if (a.absmax) {
            // |value| <= hypot(max |Re|, max |Im|), formed in FP64 (no FP32 overflow of the
            // squares); a NaN or infinite value makes the bound infinite
            float m = vbad ? INFINITY : (float)sqrt((double)vmre * vmre + (double)vmim * vmim);
            for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
            // non-negative floats order like their bit patterns; the margin matches the pre-pass
            if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax(reinterpret_cast<unsigned *>(a.absmax), __float_as_uint(m * 1.0001f));
        }
    }
}

template <typename R, int W, int LPV>
static hipError_t interp_w(const InterpLaunch &a, hipStream_t s) {
    const bool flat = a.g.flat;
    const int S = a.g.T + W;
    const size_t lds = (size_t)(flat ? 1 : W) * S * S * sizeof(cplx<R>);
#define INTERP_CASE(FL, OM)                                                         \
    if (flat == FL && a.omode == OM) {                                              \
        PFB_LAUNCH_NT((interp_kernel<R, W, LPV, FL, OM>), a.n_work, kTileThreads, lds, s, a); \
        return hipSuccess;                                                          \
    }
    INTERP_CASE(false, 0)
    INTERP_CASE(false, 1)
    INTERP_CASE(false, 2)
    INTERP_CASE(true, 0)
    INTERP_CASE(true, 1)
    INTERP_CASE(true, 2)
#undef INTERP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_interp(bool dbl, const InterpLaunch &a, hipStream_t s) {
    if (a.n_work <= 0) return hipSuccess;
    if (dbl)
        return dispatch_int<9, 16>(a.g.W, [&](auto Wc) { return interp_w<double, decltype(Wc)::value, 16>(a, s); });
    return dispatch_int<4, 8>(a.g.W, [&](auto Wc) {
        constexpr int W = decltype(Wc)::value;
        const bool flat = a.g.flat;
        const int S = a.g.T + W;
        const size_t lds = ((size_t)(flat ? 1 : W) * S * (S + kInterp4ColPad) + kInterp4Pad) * sizeof(cplx<float>);
#define INTERP4_CASE(FL, OM)                                                              \
        if (flat == FL && a.omode == OM) {                                                \
            PFB_LAUNCH_NT((interp4_kernel<W, FL, OM>), a.n_work, kTileThreads, lds, s, a); \
            return hipSuccess;                                                            \
        }
        INTERP4_CASE(false, 0)
        INTERP4_CASE(false, 1)
        INTERP4_CASE(false, 2)
        INTERP4_CASE(true, 0)
        INTERP4_CASE(true, 1)
        INTERP4_CASE(true, 2)
#undef INTERP4_CASE
        return hipErrorInvalidValue;
    });
}

template <typename R>
__global__ __launch_bounds__(kThreads) void zero_flagged_kernel(const uint32_t *idx, int64_t n, cplx<R> *vis) {
    // four indices per thread loaded before their stores; past the end the index is
    // clamped to the last flagged entry, which is then zeroed once more (no branch
    // for the compiler to sink a load into)
    constexpr int U = 4;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; e0 < n; e0 += U * stride) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = idx[min(e0 + u * stride, n - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) vis[v[u]] = cplx<R>{R(0), R(0)};
    }
}
hipError_t launch_zero_flagged(bool dbl, const uint32_t *flagged, int64_t n, void *vis, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + kThreads - 1) / kThreads;
    if (nb > 16384) nb = 16384;
    if (dbl) PFB_LAUNCH(zero_flagged_kernel<double>, nb, 0, s, flagged, n, (cplx<double> *)vis);
    else PFB_LAUNCH(zero_flagged_kernel<float>, nb, 0, s, flagged, n, (cplx<float> *)vis);
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// operator transforms (planes <-> image)
// ---------------------------------------------------------------------------
// Grid index q of image pixel i (period g): q = (i - n/2) mod g; inverse
// i = (q + n/2) mod g, valid when < n.

template <typename R>
__device__ __forceinline__ R pixel_sm1(int i, int j, const GeomDev &g) {
    const R l = R(i - g.nx / 2 + g.offx) * (R)g.cellx, m = R(j - g.ny / 2 + g.offy) * (R)g.celly;
    const R r2 = l * l + m * m;
    return -r2 / (R(1) + dev_sqrt(R(1) - r2));
}

constexpr int kRowLds = 32768;   // target LDS bytes per row-transform workgroup

// Threads of a row-transform block: one radix-8 butterfly per thread and stage
// for long rows (more waves in flight per row), at least kThreads.
template <int LOG2L> __host__ __device__ constexpr int row_threads() {
    return (1 << LOG2L) / 8 > 1024 ? 1024 : ((1 << LOG2L) / 8 < kThreads ? kThreads : (1 << LOG2L) / 8);
}
// waves per SIMD that two row-pass blocks per CU need (the register budget)
template <int LOG2L> __host__ __device__ constexpr int row_min_waves() { return row_threads<LOG2L>() / 128; }
// rows per workgroup: the largest power of two whose LDS tiles fit kRowLds
template <typename R, int LOG2L>
__host__ __device__ constexpr int rows_per_block() {
    constexpr int per = Lds<R, LOG2L>::ld * (int)sizeof(cplx<R>);
    int c = 1;
    while (2 * c * per <= kRowLds) c *= 2;
    return c;
}
// entries of the direct stage twiddle tables of a 2^LOG2L-point transform that a
// block can keep beside `other` bytes of LDS while two blocks still fit a CU
template <typename R, int LOG2L> __host__ __device__ constexpr int tw_stage_entries(size_t other) {
    constexpr size_t half = kMaxLdsBytes / 2, tab = kTwEntries * sizeof(cplx<R>);
    return other + tab >= half ? 0 : StageTab<LOG2L>::entries((int)((half - other - tab) / sizeof(cplx<R>)));
}
// bytes after a row-pass block's vectors for one tile row's occupancy flags (at
// most L / 8 tiles: tiles have at least 8 cells)
template <int LOG2L> __host__ __device__ constexpr size_t row_aux_bytes() { return ((1 << LOG2L) / 8 + 15) / 16 * 16; }
// the row passes: budget for their most rows per block
template <typename R, int LOG2L> __host__ __device__ constexpr int row_tw_se() {
    return tw_stage_entries<R, LOG2L>((size_t)rows_per_block<R, LOG2L>() * Lds<R, LOG2L>::ld * sizeof(cplx<R>) +
                                      row_aux_bytes<LOG2L>());
}
// LDS bytes of a row-pass block of C vectors
template <typename R, int LOG2L> constexpr size_t row_lds(int C) {
    return (size_t)C * (Lds<R, LOG2L>::ld * sizeof(cplx<R>)) + (kTwEntries + row_tw_se<R, LOG2L>()) * sizeof(cplx<R>) +
           row_aux_bytes<LOG2L>();
}

// Plane intermediate of the grid and degrid transforms (cropped row spectra),
// group-major: column iy = g CG + c of uv row u of plane (bb, j) sits at
// T[(((bb nwmax + j) G + g) gx + u) CG + c], G = ceil(ny / CG), CG complex values
// in 64 bytes.  The row passes store and load 64-byte pieces (neighbouring rows
// complete the lines); the gx rows of a group are one contiguous block for the
// column passes, whose CG / C blocks per group share it through one XCD's L2
// (64 bytes measured faster overall than 32 or 128).
template <typename R> __host__ __device__ constexpr int plane_cg() { return 64 / (int)sizeof(cplx<R>); }
template <typename R> __device__ __forceinline__ size_t plane_at(const XformArgs &a, size_t plane, int u, int iy) {
    constexpr int CG = plane_cg<R>();
    const int G = (a.g.ny + CG - 1) / CG;
    return ((plane * G + (size_t)(iy / CG)) * a.g.gx + u) * CG + (iy & (CG - 1));
}
int plane_group_cols(bool dbl) { return dbl ? plane_cg<double>() : plane_cg<float>(); }

// Blocks go to the eight XCDs in turn (block i on XCD i mod 8).  For a grid that
// is a multiple of 8 this returns the logical block of block i such that each XCD
// runs one contiguous range of logical blocks: neighbouring rows of the row
// passes then share an XCD and their partial cache lines of the group-major
// layout meet in its L2.
__device__ __forceinline__ int xcd_block(int i, int n) {
    return (n & 7) ? i : (i & 7) * (n >> 3) + (i >> 3);
}

// G1: inverse row DFT of every plane row, keeping the ny cropped outputs.
template <typename R, int LOG2L>
__global__ __launch_bounds__(row_threads<LOG2L>(), row_min_waves<LOG2L>()) void g1_rows_kernel(XformArgs a, int C) {
    constexpr int L = 1 << LOG2L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + row_tw_se<R, LOG2L>();
    const TwTab<R> tt = tw_fill<R, row_threads<LOG2L>(), LOG2L, row_tw_se<R, LOG2L>()>(
        twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    const int ld = Lds<R, LOG2L>::ld;
    const int gx = a.g.gx;
    // block: C consecutive rows of a listed tile row (one that holds occupied tiles)
    const int per = a.g.T / C;
    const int lb = xcd_block(blockIdx.x, gridDim.x);   // rows of a tile row on one XCD
    const int e = a.occ_list[lb / per];   // (band nwmax + plane) ntx + tile row
    const int pj = e / a.g.ntx;
    const int j = pj % a.g.nwmax, bb = pj / a.g.nwmax - a.band0;
    const int row0 = (e - pj * a.g.ntx) * a.g.T + (lb % per) * C;
    const size_t plane = (size_t)bb * a.g.nwmax + j;
    const cplx<R> *src = reinterpret_cast<const cplx<R> *>(a.planes) + (plane * gx + (size_t)row0) * L;
    cplx<R> *dst = reinterpret_cast<cplx<R> *>(a.t1);
    // tiles of these rows that hold spread values (the rest of the plane is zero
    // and is not read)
    const int lgT = __builtin_ctz(a.g.T), nty = a.g.nty;   // tiles are powers of two
    // the C rows lie in one tile row: its flags go to LDS first, so that the row
    // loads do not wait on flag loads
    const uint8_t *occ = a.occ + ((size_t)pj * a.g.ntx + (row0 >> lgT)) * nty;
    uint8_t *occ_l = reinterpret_cast<uint8_t *>(buf + C * ld);
    for (int k = threadIdx.x; k < nty; k += row_threads<LOG2L>()) occ_l[k] = occ[k];
    __syncthreads();
    const int ny = a.g.ny;
    // output k of the row DFT is cropped column iy = k + ny / 2 (mod L), kept if iy < ny
    row_fft<R, true, LOG2L, row_threads<LOG2L>(), true, fuse_first8<LOG2L>(), 8>(
        buf, C, ld, tt, a.log2_lmax - LOG2L,
        [&](int c, int r) -> cplx<R> {
            cplx<R> v{R(0), R(0)};
            if (occ_l[r >> lgT]) v = src[(size_t)c * L + r];
            return v;
        },
        InPlain{}, OutNoFetch{},
        [&](int c, int k, const cplx<R> &v, NoRaw) {
            const int iy = (k + ny / 2) & (L - 1);
            if (iy < ny) dst[plane_at<R>(a, plane, row0 + c, iy)] = v;
        });
}

// D3: forward row DFT of the ny placed inputs of each row (the rows the degrid
// column pass wrote: tile rows with needed tiles), full output to the plane.
template <typename R, int LOG2L>
__global__ __launch_bounds__(row_threads<LOG2L>(), row_min_waves<LOG2L>()) void d3_rows_kernel(XformArgs a, int C) {
    constexpr int L = 1 << LOG2L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + row_tw_se<R, LOG2L>();
    const TwTab<R> tt = tw_fill<R, row_threads<LOG2L>(), LOG2L, row_tw_se<R, LOG2L>()>(
        twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    const int ld = Lds<R, LOG2L>::ld;
    const int gx = a.g.gx, ny = a.g.ny;
    // block: C consecutive rows of a listed tile row (one with tiles the interpolation reads)
    const int per = a.g.T / C;
    const int lb = xcd_block(blockIdx.x, gridDim.x);   // rows of a tile row on one XCD
    const int e = a.need_list[lb / per];   // (band nwmax + plane) ntx + tile row
    const int pj = e / a.g.ntx;
    const int j = pj % a.g.nwmax, bb = pj / a.g.nwmax - a.band0;
    const int row0 = (e - pj * a.g.ntx) * a.g.T + (lb % per) * C;
    const size_t plane = (size_t)bb * a.g.nwmax + j;
    const cplx<R> *src = reinterpret_cast<const cplx<R> *>(a.t1);
    cplx<R> *dst = reinterpret_cast<cplx<R> *>(a.planes) + (plane * gx + (size_t)row0) * L;
    // only tiles the interpolation may read are written
    const int lgT = __builtin_ctz(a.g.T), nty = a.g.nty;   // tiles are powers of two
    // the C rows lie in one tile row; its flags in LDS (read after the transform's
    // barriers) keep flag loads out of the store loop
    const uint8_t *need = a.need + ((size_t)pj * a.g.ntx + (row0 >> lgT)) * nty;
    uint8_t *need_l = reinterpret_cast<uint8_t *>(buf + C * ld);
    for (int k = threadIdx.x; k < nty; k += row_threads<LOG2L>()) need_l[k] = need[k];
    // input r of the row DFT is cropped column iy = r + ny / 2 (mod L), zero if iy >= ny
    row_fft<R, false, LOG2L, row_threads<LOG2L>(), true, true>(
        buf, C, ld, tt, a.log2_lmax - LOG2L,
        [&](int c, int r) -> cplx<R> {
            const int iy = (r + ny / 2) & (L - 1);
            cplx<R> v{R(0), R(0)};
            if (iy < ny) v = src[plane_at<R>(a, plane, row0 + c, iy)];
            return v;
        },
        InPlain{}, OutNoFetch{},
        [&](int c, int k, const cplx<R> &v, NoRaw) {
            if (need_l[k >> lgT]) dst[(size_t)c * L + k] = v;
        });
}

// Column passes of the w-plane transforms: for every column of the cropped row
// spectra, the gx-point DFT over u between the uv rows and the image rows
// i = 0 .. nx - 1, in one pass per plane with the plane loop inside the block.
// With N = gx / 2, w = exp(-2 pi i / gx) and the image centred on the grid
// origin (DFT index n = i - nx / 2, hx = nx / 2), nx <= N lets the gx-point
// transforms split into N-point ones over even and odd u:
//   grid   F(i) = sum_u G[u] w^(-u n) = E[i] + w^-i O[i],
//          E, O = inverse N-point DFTs of G'[u] = G[u] w^(u hx) over even / odd u;
//   degrid X[2k' + p] = w^(-(2k' + p) hx) DFT_N(x[i] w^(p i))[k']   (p = 0, 1),
// so one column needs N complex values of LDS at a time.  The grid pass reads
// only the rows of tile rows with occupied tiles (the others are zero and were
// not written) and accumulates Re(F_j(i) e^(2 pi i w_j (n_i - 1 - sc))) over the
// planes in registers before the grid correction; the degrid pass keeps the
// corrected image column in registers and writes, for every plane, only the
// rows of tile rows the forward row pass reads.
template <typename R, int LOG2N, int C> struct WCols {
    static constexpr int N = 1 << LOG2N;
    static constexpr int NT0 = C * N / 8;   // one radix-8 butterfly per thread and stage
    static constexpr int NT = NT0 < 64 ? 64 : NT0;
    static_assert(NT0 <= 1024, "at most 1024 threads per block");
    static constexpr int R0 = FftPlan<LOG2N>::radix(0);
    static constexpr int ITER = (C * (N / R0) + NT - 1) / NT;   // innermost-stage items per thread
    // the transform buffer, the twiddle tables and two per-thread arrays of 8 values
    // that live across the plane loop (kept in LDS, not in registers)
    // plus two buffers of a plane's tile-row flags (at most gx / 8 = N / 4 tile rows)
    static constexpr size_t other =
        (size_t)C * Lds<R, LOG2N>::ld * sizeof(cplx<R>) + 2 * 8 * (size_t)NT * sizeof(R) + 2 * (size_t)(N / 4);
    static constexpr int SE = tw_stage_entries<R, LOG2N>(other);
    static constexpr size_t lds = other + (kTwEntries + SE) * sizeof(cplx<R>);
};
// columns per block: the most (up to a whole group) whose C x N block spans at
// most 1024 threads and 64 KiB of LDS
template <typename R, int LG> constexpr int wcols_c() {
    constexpr int N = 1 << LG;
    constexpr int a = 4096 / N, b = (int)(65536 / ((size_t)N * sizeof(cplx<R>)));
    constexpr int c = a < b ? a : b;
    return c < 1 ? 1 : (c > plane_cg<R>() ? plane_cg<R>() : c);
}

// Blocks go to the XCDs in turn (block i on XCD i mod 8); the CG / C blocks of one
// column group get indices that share i mod 8 and follow each other, so they run
// together on one XCD and read (or write) the group's 128-byte lines through its L2.
struct WColsBlock {
    int g, sub, bb;
    bool ok;
};
template <int NSUB> __device__ __forceinline__ WColsBlock wcols_block(int n_bb, int G) {
    const int xcd = blockIdx.x & 7, jb = blockIdx.x >> 3;
    const int gi = (jb / NSUB) * 8 + xcd;
    return WColsBlock{gi % G, jb % NSUB, gi / G, gi < n_bb * G};
}

template <typename R, int LOG2N, int C>
__global__ __launch_bounds__((WCols<R, LOG2N, C>::NT)) void wgrid_cols_kernel(XformArgs a) {
    using K = WCols<R, LOG2N, C>;
    using LD = Lds<R, LOG2N>;
    using P = FftPlan<LOG2N>;
    constexpr int N = K::N, NT = K::NT, S = P::NSTAGE, M = N / 8, R0 = K::R0, IT = K::ITER;
    constexpr int CG = plane_cg<R>(), ld = LD::ld;
    static_assert(S >= 2 && P::radix(S - 1) == 8, "columns of at least 16 points");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + K::SE;
    const TwTab<R> tt = tw_fill<R, NT, LOG2N, K::SE>(twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    const int gx = a.g.gx, nx = a.g.nx, ny = a.g.ny, hx = nx / 2;
    const int G = (ny + CG - 1) / CG;
    const WColsBlock wb = wcols_block<CG / C>(a.n_bb, G);
    if (!wb.ok) return;
    const int b = a.band0 + wb.bb;
    const BandDev bd = a.bands[b];
    const int nw = a.g.flat ? 1 : bd.nw;
    const int col0 = wb.g * CG + wb.sub * C;
    const int shg = a.log2_lmax - (LOG2N + 1), shn = a.log2_lmax - LOG2N;
    const int lgT = __builtin_ctz(a.g.T);
    // gx = 2 nx (power-of-two sides): G'[u] = G[u] (-i)^u, so the even half's
    // transform is that of G[2u'] shifted by N / 2 and the odd half's also times -i:
    // pixel i comes from natural index i ^ N / 2 and the odd half's factor is
    // w^-(i - N / 2); no product on the loaded values
    const bool qs = 4 * hx == gx;
    const int hs = qs ? N / 2 : 0;
    // first stage: thread (c, jr) owns the butterfly of rows u' = jr + t M (t < 8)
    const int c = threadIdx.x % C, jr = threadIdx.x / C;
    const bool own = jr < M && col0 + c < ny;
    // innermost stage: item (it, t) is position gq R0 + t of column cc, natural index i;
    // its n - 1 - sc and accumulator sit in LDS slot (it R0 + t) NT + thread
    cplx<R> ev[IT][R0];
    R *const svl = reinterpret_cast<R *>(buf + C * ld);
    R *const accl = svl + 8 * NT;
    const R sc = (R)bd.sc;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int id = threadIdx.x + it * NT;
        const int cc = id / (N / R0), gq = id - cc * (N / R0);
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int i = dit_inv<LOG2N>(gq * R0 + t) ^ hs;
            const int sl = (it * R0 + t) * NT + threadIdx.x;
            accl[sl] = R(0);
            svl[sl] = (!a.g.flat && id < C * (N / R0) && i < nx && col0 + cc < ny) ? pixel_sm1<R>(i, col0 + cc, a.g) - sc
                                                                                    : R(0);
        }
    }
    uint8_t *const flb = reinterpret_cast<uint8_t *>(accl + 8 * NT);   // two buffers of ntx flags
    for (int j = 0; j < nw; ++j) {
        // the plane's tile-row flags go to LDS, so that the row loads do not wait on flag loads
        const uint8_t *orow = a.occ_row + ((size_t)b * a.g.nwmax + j) * a.g.ntx;
        uint8_t *const fl = flb + (j & 1) * (N / 4);
        int any = 0;
        for (int k = threadIdx.x; k < a.g.ntx; k += NT) {
            fl[k] = orow[k];
            any |= orow[k];
        }
        if (!__syncthreads_or(any)) continue;   // (also orders the twiddle table and the last plane's LDS reads)
        const cplx<R> *T = reinterpret_cast<const cplx<R> *>(a.t1) +
                           (((size_t)wb.bb * a.g.nwmax + j) * G + wb.g) * (size_t)gx * CG + wb.sub * C;
        const R wj = (R)(bd.w0 + j * bd.dw);
#pragma unroll 1
        for (int p = 0; p < 2; ++p) {
            // inverse N-point DFT of the even (p = 0) or odd (p = 1) rows by decimation in
            // frequency: the first stage straight from HBM, output i ends at the DIT position of i
            if (own) {
                cplx<R> v[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {   // all loads first
                    const int u = 2 * (jr + t * M) + p;
                    v[t] = cplx<R>{R(0), R(0)};
                    if (fl[u >> lgT]) v[t] = T[(size_t)u * CG + c];
                }
                if (!qs) {
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int u = 2 * (jr + t * M) + p;
                        v[t] = v[t] * twiddle<R, false>(tt, ((u * hx) & (gx - 1)) << shg);
                    }
                }
                dft_small<R, true, 8>(v);
                stage_twiddles<R, true, 8>(v, tt, jr << shn);
                cplx<R> *vb = buf + c * ld + LD::pad(jr);
#pragma unroll
                for (int t = 0; t < 8; ++t) vb[LD::pad(t * M)] = v[t];
            } else if (jr < M) {
                cplx<R> *vb = buf + c * ld + LD::pad(jr);
#pragma unroll
                for (int t = 0; t < 8; ++t) vb[LD::pad(t * M)] = cplx<R>{R(0), R(0)};
            }
            __syncthreads();
            {
                int m = M;
#pragma unroll
                for (int st = S - 2; st >= 1; --st) {   // middle stages, radix 8
                    m /= 8;
                    dif_stage<R, true, 8, LOG2N, NT>(buf, C, ld, m, tt, shn);
                    __syncthreads();
                }
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int id = threadIdx.x + it * NT;
                if (id >= C * (N / R0)) continue;
                const int cc = id / (N / R0), gq = id - cc * (N / R0);
                const cplx<R> *vb = buf + cc * ld + LD::pad(gq * R0);
                cplx<R> v[R0];
#pragma unroll
                for (int t = 0; t < R0; ++t) v[t] = vb[LD::pad(t)];
                dft_small<R, true, R0>(v);
#pragma unroll
                for (int t = 0; t < R0; ++t) {
                    if (p == 0) {
                        ev[it][t] = v[t];
                    } else {
                        const int i = dit_inv<LOG2N>(gq * R0 + t) ^ hs;
                        const int sl = (it * R0 + t) * NT + threadIdx.x;
                        const int e = qs ? (i + gx - N / 2) & (gx - 1) : i;
                        const cplx<R> y = ev[it][t] + v[t] * twiddle<R, true>(tt, e << shg);
                        if (a.g.flat) {
                            accl[sl] += y.re;
                        } else {
                            const cplx<R> ph = cis_cycles<R>(wj * svl[sl]);
                            accl[sl] += y.re * ph.re - y.im * ph.im;
                        }
                    }
                }
            }
            if (p == 0) __syncthreads();   // the odd half overwrites the buffer
        }
    }
    R *img = reinterpret_cast<R *>(a.image_out) + (size_t)b * nx * ny;
    const R *corr2d = reinterpret_cast<const R *>(a.corr2d);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int id = threadIdx.x + it * NT;
        const int cc = id / (N / R0), gq = id - cc * (N / R0);
        const int col = col0 + cc;
        if (id >= C * (N / R0) || col >= ny) continue;
        // the correction factors' loads first (corr2d, or corr_x[i] times corr_y[col])
        R cf[R0];
        const R cy = corr2d ? R(1) : reinterpret_cast<const R *>(a.corr_y)[col];
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int i = dit_inv<LOG2N>(gq * R0 + t) ^ hs;
            cf[t] = R(0);
            if (i < nx)
                cf[t] = corr2d ? corr2d[(size_t)b * nx * ny + (size_t)i * ny + col] : reinterpret_cast<const R *>(a.corr_x)[i];
        }
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int i = dit_inv<LOG2N>(gq * R0 + t) ^ hs;
            if (i >= nx) continue;
            R v = accl[(it * R0 + t) * NT + threadIdx.x] * (cf[t] * cy);
            if (a.zero_edge && (i == 0 || col == 0)) v = R(0);
            img[(size_t)i * ny + col] = v;
        }
    }
}

template <typename R, int LOG2N, int C>
__global__ __launch_bounds__((WCols<R, LOG2N, C>::NT)) void wdegrid_cols_kernel(XformArgs a) {
    using K = WCols<R, LOG2N, C>;
    using LD = Lds<R, LOG2N>;
    using P = FftPlan<LOG2N>;
    constexpr int N = K::N, NT = K::NT, S = P::NSTAGE, M = N / 8, R0 = K::R0, IT = K::ITER;
    constexpr int CG = plane_cg<R>(), ld = LD::ld;
    static_assert(S >= 2 && P::radix(S - 1) == 8, "columns of at least 16 points");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + K::SE;
    const TwTab<R> tt = tw_fill<R, NT, LOG2N, K::SE>(twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    const int gx = a.g.gx, nx = a.g.nx, ny = a.g.ny, hx = nx / 2;
    const int G = (ny + CG - 1) / CG;
    const WColsBlock wb = wcols_block<CG / C>(a.n_bb, G);
    if (!wb.ok) return;
    const int b = a.band0 + wb.bb;
    const BandDev bd = a.bands[b];
    const int nw = a.g.flat ? 1 : bd.nw;
    const int col0 = wb.g * CG + wb.sub * C;
    const int shg = a.log2_lmax - (LOG2N + 1), shn = a.log2_lmax - LOG2N;
    const int lgT = __builtin_ctz(a.g.T);
    // gx = 2 nx (power-of-two sides): w^(-u hx) = i^u = (-1)^k' i^p for u = 2k' + p,
    // so position m of the transforms takes image row m ^ N / 2, the odd half's
    // input factor becomes w^(i - N / 2), and the outputs need no product
    const bool qs = 4 * hx == gx;
    const int hs = qs ? N / 2 : 0;
    // first stage: thread (c, jr) owns positions jr + t M (t < 8), image rows
    // (jr + t M) ^ hs, of column col
    const int c = threadIdx.x % C, jr = threadIdx.x / C;
    const int col = col0 + c;
    const bool own = jr < M;
    // the corrected image value and n - 1 - sc of row t of the thread: LDS slot t NT + thread
    R *const xrl = reinterpret_cast<R *>(buf + C * ld);
    R *const svl = xrl + 8 * NT;
    const R sc = (R)bd.sc;
    {
        // loads first: image values and correction factors (corr2d, or corr_x[i] times corr_y[col])
        const R *corr2d = reinterpret_cast<const R *>(a.corr2d);
        const bool colok = own && col < ny;
        const R cy = (corr2d || !colok) ? R(1) : reinterpret_cast<const R *>(a.corr_y)[col];
        R xs[8], cf[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int i = (jr + t * M) ^ hs;
            xs[t] = cf[t] = R(0);
            if (colok && i < nx) {
                const size_t pix = (size_t)b * nx * ny + (size_t)i * ny + col;
                xs[t] = reinterpret_cast<const R *>(a.image_in)[pix];
                cf[t] = corr2d ? corr2d[pix] : reinterpret_cast<const R *>(a.corr_x)[i];
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int i = (jr + t * M) ^ hs;
            R s = R(0);
            if (colok && i < nx && !a.g.flat) s = pixel_sm1<R>(i, col, a.g) - sc;
            xrl[t * NT + threadIdx.x] = xs[t] * (cf[t] * cy);
            svl[t * NT + threadIdx.x] = s;
        }
    }
    uint8_t *const flb = reinterpret_cast<uint8_t *>(svl + 8 * NT);   // two buffers of ntx flags
    for (int j = 0; j < nw; ++j) {
        // the plane's tile-row flags go to LDS (two buffers: the last plane's stores may
        // still read the other), so that the stores do not wait on flag loads
        const uint8_t *nrow = a.need_row + ((size_t)b * a.g.nwmax + j) * a.g.ntx;
        uint8_t *const fl = flb + (j & 1) * (N / 4);
        int any = 0;
        for (int k = threadIdx.x; k < a.g.ntx; k += NT) {
            fl[k] = nrow[k];
            any |= nrow[k];
        }
        if (!__syncthreads_or(any)) continue;   // (also orders the twiddle table and the last plane's LDS reads)
        cplx<R> *T = reinterpret_cast<cplx<R> *>(a.t1) +
                     (((size_t)wb.bb * a.g.nwmax + j) * G + wb.g) * (size_t)gx * CG + wb.sub * C;
        const R wj = (R)(bd.w0 + j * bd.dw);
        cplx<R> pv[8];   // x e^(-2 pi i w_j (n - 1 - sc))
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const R xv = xrl[t * NT + threadIdx.x];
            pv[t] = a.g.flat ? cplx<R>{xv, R(0)} : conj(cis_cycles<R>(wj * svl[t * NT + threadIdx.x])) * xv;
        }
#pragma unroll 1
        for (int p = 0; p < 2; ++p) {
            // forward N-point DFT of x w^(p i) by decimation in frequency: the first stage
            // from registers, X[k'] ends at the DIT position of k'.  The odd half's factor
            // at position jr + t M is w^jr exp(-2 pi i t / 16), negated for t >= 4 when the
            // rows are shifted (w^N = -1)
            if (own) {
                cplx<R> v[8];
                const cplx<R> wj = twiddle<R, false>(tt, jr << shg);
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    cplx<R> f = wj * root16<R>(t);
                    if (qs && t >= 4) f = cplx<R>{-f.re, -f.im};
                    v[t] = p == 0 ? pv[t] : pv[t] * f;
                }
                dft_small<R, false, 8>(v);
                stage_twiddles<R, false, 8>(v, tt, jr << shn);
                cplx<R> *vb = buf + c * ld + LD::pad(jr);
#pragma unroll
                for (int t = 0; t < 8; ++t) vb[LD::pad(t * M)] = v[t];
            }
            __syncthreads();
            {
                int m = M;
#pragma unroll
                for (int st = S - 2; st >= 1; --st) {   // middle stages, radix 8
                    m /= 8;
                    dif_stage<R, false, 8, LOG2N, NT>(buf, C, ld, m, tt, shn);
                    __syncthreads();
                }
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int id = threadIdx.x + it * NT;
                if (id >= C * (N / R0)) continue;
                const int cc = id / (N / R0), gq = id - cc * (N / R0);
                if (col0 + cc >= ny) continue;
                const cplx<R> *vb = buf + cc * ld + LD::pad(gq * R0);
                cplx<R> v[R0];
#pragma unroll
                for (int t = 0; t < R0; ++t) v[t] = vb[LD::pad(t)];
                dft_small<R, false, R0>(v);
#pragma unroll
                for (int t = 0; t < R0; ++t) {
                    const int u = 2 * dit_inv<LOG2N>(gq * R0 + t) + p;
                    if (fl[u >> lgT])
                        T[(size_t)u * CG + cc] = qs ? v[t] : v[t] * twiddle<R, true>(tt, ((u * hx) & (gx - 1)) << shg);
                }
            }
            if (p == 0) __syncthreads();   // the odd half overwrites the buffer
        }
    }
}

template <typename R, bool GRID>
static hipError_t wcols_launch(const XformArgs &a, hipStream_t s) {
    return dispatch_int<4, 13>(__builtin_ctz(a.g.gx) - 1, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        if constexpr (sizeof(R) == 8 && LG > 12) {
            return hipErrorInvalidValue;   // FP64 plane rows stop at 8192 points
        } else {
            constexpr int C = wcols_c<R, LG>();
            constexpr int CG = plane_cg<R>();
            using K = WCols<R, LG, C>;
            const int G = (a.g.ny + CG - 1) / CG;
            const int nb = ((a.n_bb * G + 7) / 8) * 8 * (CG / C);
            if (GRID) PFB_LAUNCH_NT((wgrid_cols_kernel<R, LG, C>), nb, K::NT, K::lds, s, a);
            else PFB_LAUNCH_NT((wdegrid_cols_kernel<R, LG, C>), nb, K::NT, K::lds, s, a);
            return hipSuccess;
        }
    });
}

template <typename R>
static hipError_t grid_xform_t(const XformArgs &a, hipStream_t s) {
    const int lgy = __builtin_ctz(a.g.gy);
    hipError_t e = dispatch_int<5, 14>(lgy, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        const int C = std::min(rows_per_block<R, LG>(), a.g.T);
        const size_t lds = row_lds<R, LG>(C);
        const int64_t nb = (int64_t)a.n_occ_list * (a.g.T / C);
        if (nb > 0) PFB_LAUNCH_NT((g1_rows_kernel<R, LG>), nb, row_threads<LG>(), lds, s, a, C);
        return hipSuccess;
    });
    if (e != hipSuccess) return e;
    return wcols_launch<R, true>(a, s);
}

template <typename R>
static hipError_t degrid_xform_t(const XformArgs &a, hipStream_t s) {
    hipError_t e = wcols_launch<R, false>(a, s);
    if (e != hipSuccess) return e;
    const int lgy = __builtin_ctz(a.g.gy);
    return dispatch_int<5, 14>(lgy, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        const int C2 = std::min(rows_per_block<R, LG>(), a.g.T);
        const size_t lds = row_lds<R, LG>(C2);
        const int64_t nb = (int64_t)a.n_need_list * (a.g.T / C2);
        if (nb > 0) PFB_LAUNCH_NT((d3_rows_kernel<R, LG>), nb, row_threads<LG>(), lds, s, a, C2);
        return hipSuccess;
    });
}

hipError_t launch_grid_xform(bool dbl, const XformArgs &a, hipStream_t s) {
    return dbl ? grid_xform_t<double>(a, s) : grid_xform_t<float>(a, s);
}
hipError_t launch_degrid_xform(bool dbl, const XformArgs &a, hipStream_t s) {
    return dbl ? degrid_xform_t<double>(a, s) : degrid_xform_t<float>(a, s);
}

// ---------------------------------------------------------------------------
// PSF convolution on the 2nx x 2ny zero-padded grid
// ---------------------------------------------------------------------------


// Offset (in complex values, within a band's lx ldh area of t1c) of the column
// pass's output in image mode: the upper half, free since nx <= lx / 2.
__device__ __forceinline__ size_t conv_out_off(const ConvArgs &a) { return (size_t)(a.lx / 2) * a.ldh; }

// S1: forward row DFT (length 2ny) of real rows, keeping the half spectrum k = 0..ny.
//   in_mode CONV_IN_X      : row i of x (ny values, zero padded)
//           CONV_IN_CG_P   : p = r + beta p, written back, then transformed
//           CONV_IN_SCALED : x * scale
//   psfhat mode (nrows = 2nx): row i of the PSF rolled by (nx, ny)
// Two real rows share one complex transform: rows 2c and 2c + 1 of the block
// are the real and imaginary parts of vector c, and their half spectra come
// out as X_a[k] = (Z[k] + conj Z[L - k]) / 2, X_b[k] = (Z[k] - conj Z[L - k]) / 2i.
// C vectors (2C rows) per block.
template <typename R, int LOG2L, int IN>
__global__ __launch_bounds__(row_threads<LOG2L>(), row_min_waves<LOG2L>()) void s1_kernel(ConvArgs a, const R *x, R *auxp, int nrows, int C, int psf) {
    constexpr int L = 1 << LOG2L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + row_tw_se<R, LOG2L>();
    const TwTab<R> tt = tw_fill<R, row_threads<LOG2L>(), LOG2L, row_tw_se<R, LOG2L>()>(
        twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    const int ld = Lds<R, LOG2L>::ld;
    const int nx = a.nx, ny = a.ny;
    const int ngrp = nrows / (2 * C);
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int ig = lb % ngrp;
    const int b = lb / ngrp;
    R bscale = R(1);
    if (IN == CONV_IN_CG_P) bscale = (R)a.scal[b * 8 + S_BETA];
    if (IN == CONV_IN_SCALED) bscale = (R)a.scal[b * 8 + S_SCALE];
    // inputs r of rows i = ig 2C + 2c and i + 1 (one complex vector): loads first,
    // then the value (and the CG direction update p = x + beta p, stored back);
    // the PSF (psf = 1, CONV_IN_X only) is read with its offsets rolled to the origin
    struct RawP {
        R x0, x1, p0, p1;
    };
    row_fft<R, false, LOG2L, row_threads<LOG2L>(), false, fuse_first8<LOG2L>()>(
        buf, C, ld, tt, a.log2_lmax - LOG2L,
        [&](int c, int r) {
            const int i = ig * 2 * C + 2 * c;
            if constexpr (IN == CONV_IN_CG_P) {
                RawP raw{R(0), R(0), R(0), R(0)};
                if (r < ny) {
                    const size_t pix = ((size_t)b * nx + i) * ny + r;
                    raw = RawP{x[pix], x[pix + ny], auxp[pix], auxp[pix + ny]};
                }
                return raw;
            } else {
                cplx<R> raw{R(0), R(0)};
                if (psf) {
                    // grid index i holds offset di = i (first half) or i - lx (second half) of
                    // the PSF; offsets outside [-nx, nx) x [-ny, ny) are zero
                    const int dj = r < a.ly / 2 ? r : r - a.ly;
                    if (dj >= -ny && dj < ny) {
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int di = i + h < a.lx / 2 ? i + h : i + h - a.lx;
                            if (di >= -nx && di < nx) {
                                const R v = x[((size_t)b * 2 * nx + di + nx) * 2 * ny + dj + ny];
                                if (h) raw.im = v;
                                else raw.re = v;
                            }
                        }
                    }
                } else if (r < ny) {
                    const size_t pix = ((size_t)b * nx + i) * ny + r;
                    raw = cplx<R>{x[pix], x[pix + ny]};
                }
                return raw;
            }
        },
        [&](int c, int r, const auto &raw) -> cplx<R> {
            if constexpr (IN == CONV_IN_CG_P) {
                const cplx<R> v{raw.x0 + bscale * raw.p0, raw.x1 + bscale * raw.p1};
                if (r < ny) {
                    const size_t pix = ((size_t)b * nx + ig * 2 * C + 2 * c) * ny + r;
                    auxp[pix] = v.re;
                    auxp[pix + ny] = v.im;
                }
                return v;
            } else if constexpr (IN == CONV_IN_SCALED) {
                return raw * bscale;
            } else {
                return raw;
            }
        },
        OutNoFetch{}, [](int, int, const cplx<R> &, NoRaw) {});
    // group-major store: frequency k = g CG + cc of row i at (g nrows + i) CG + cc
    cplx<R> *t1 = reinterpret_cast<cplx<R> *>(a.t1c) + (size_t)b * a.lx * a.ldh;
    const int lgc = __builtin_ctz(a.cgc), cmask = a.cgc - 1;
    constexpr int NK = L / 2 + 1;   // frequencies 0 .. L/2 of a real row
    for (int id = threadIdx.x; id < C * NK; id += row_threads<LOG2L>()) {
        const int c = id / NK, k = id - c * NK;
        const cplx<R> z = buf[c * ld + Lds<R, LOG2L>::pad(k)];
        const cplx<R> zc = conj(buf[c * ld + Lds<R, LOG2L>::pad((L - k) & (L - 1))]);
        const size_t o = (((size_t)(k >> lgc) * nrows + ig * 2 * C + 2 * c) << lgc) + (k & cmask);
        t1[o] = cplx<R>{(z.re + zc.re) * R(0.5), (z.im + zc.im) * R(0.5)};
        t1[o + a.cgc] = cplx<R>{(z.im - zc.im) * R(0.5), (zc.re - z.re) * R(0.5)};
    }
}

// Group-major half-spectrum layout of the convolution's intermediate: frequency
// column k = g C + c of row i sits at T[band][(g rows + i) C + c] (rows = nx, or
// 2nx for the PSF; C values = one 128-byte line), so the rows of a group of C
// columns form one contiguous block (the column pass reads and writes whole
// blocks) and the row passes store and load whole lines.  The PSF spectrum uses
// the same groups: psfhat[band][(g 2 + p) nx + k'][c] holds frequency 2k' + p of
// column g C + c.

// Column pass: for every column (nx complex values of the row spectra; rows nx ..
// 2nx - 1 of the zero-padded grid are zero) the 2nx-point DFT, the product with
// the PSF spectrum, the inverse DFT and the crop to rows 0 .. nx - 1, in one pass.
// With N = nx and w = exp(-2 pi i / 2N) the zero padding splits the 2N-point
// transforms into N-point ones:
//   X[2k'] = DFT_N(x)[k'],  X[2k' + 1] = DFT_N(x[r] w^r)[k'],
//   y[n] = IDFT_N(H X)_even[n] + w^-n IDFT_N(H X)_odd[n]   (n < N; unnormalised),
// so one column needs N complex values of LDS at a time (C columns per block).
// PSF mode: the 2N rows of the rolled PSF (x[r] and x[r + N] both present):
//   X[2k'] = DFT_N(x[r] + x[r + N]),  X[2k' + 1] = DFT_N((x[r] - x[r + N]) w^r),
// and the real parts are stored into psfhat.
template <typename R, int LOG2N, int C> struct ConvCols {
    static constexpr int N = 1 << LOG2N;
    static constexpr int NT0 = C * N / 8;   // one radix-8 butterfly per thread and stage
    static constexpr int NT = NT0 < 64 ? 64 : NT0;
    static_assert(NT0 <= 1024, "at most 1024 threads per block");
    static constexpr int SE = tw_stage_entries<R, LOG2N>((size_t)C * Lds<R, LOG2N>::ld * sizeof(cplx<R>));
    static constexpr size_t lds = (size_t)C * Lds<R, LOG2N>::ld * sizeof(cplx<R>) + (kTwEntries + SE) * sizeof(cplx<R>);
};

// A block transforms C of the CG columns of a group (CG / C blocks per group).
// Blocks are dispatched to the eight XCDs in turn (block i on XCD i mod 8), so
// the blocks of one group get indices that share i mod 8 and follow each other
// there: they run at the same time on one XCD and read the group's rows through
// its L2 (each block reads C of every CG contiguous values).
template <typename R, int LOG2N, int C, int CG, bool PSF>
__global__ __launch_bounds__((ConvCols<R, LOG2N, C>::NT)) void conv_cols_kernel(ConvArgs a) {
    using K = ConvCols<R, LOG2N, C>;
    using LD = Lds<R, LOG2N>;
    using P = FftPlan<LOG2N>;
    constexpr int N = K::N, NT = K::NT;
    constexpr int S = P::NSTAGE;
    static_assert(S >= 2 && P::radix(S - 1) == 8, "columns of at least 16 points");
    constexpr int M = N / 8;          // span of the outermost (radix-8) stage
    constexpr int R0 = P::radix(0);   // radix of the innermost stage (span 1)
    constexpr int NSUB = CG / C;
    constexpr int ld = LD::ld;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + K::SE;
    const TwTab<R> tt = tw_fill<R, NT, LOG2N, K::SE>(twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    const int G = (a.ly / 2 + CG) / CG;   // groups of the ly / 2 + 1 columns
    const int xcd = blockIdx.x & 7, jb = blockIdx.x >> 3;
    const int sub = jb % NSUB, gi = (jb / NSUB) * 8 + xcd;
    if (gi >= a.n_band * G) return;   // the grid is padded to whole rounds of eight
    const int g = gi % G, b = gi / G;
    if (g * CG + sub * C > a.ly / 2) return;   // columns of the last group past the half spectrum
    const size_t boff = (size_t)b * a.lx * a.ldh;
    const int nin = PSF ? 2 * N : a.nx;   // rows with data; the rest of the padded column is zero
    // a group holds the rows the row pass wrote: all 2N of the PSF, the image's nx otherwise
    const cplx<R> *T = reinterpret_cast<const cplx<R> *>(a.t1c) + boff + (size_t)g * (PSF ? 2 * N : a.nx) * CG + sub * C;
    // output (image mode): the same group layout in the upper half of the band's area,
    // which the image's nx <= lx / 2 rows leave free
    cplx<R> *Y = reinterpret_cast<cplx<R> *>(a.t1c) + boff + conv_out_off(a) + (size_t)g * a.nx * CG + sub * C;
    R *H = reinterpret_cast<R *>(a.psfhat) + boff + (size_t)g * 2 * N * CG + sub * C;
    const int sh2n = a.log2_lmax - (LOG2N + 1);   // table step of w = exp(-2 pi i / 2N)
    const int shn = a.log2_lmax - LOG2N;
    // outermost stage: thread (c, j) owns the butterfly of rows j + t M (t < 8) of
    // column c; consecutive threads read consecutive values of T
    const int c = threadIdx.x % C, j = threadIdx.x / C;
    const bool own = j < M;
    cplx<R> ev[8];   // the even half's outputs y_e[j + t M], kept for the odd half
    cplx<R> xin[8];  // image mode: the thread's inputs, read once for both halves
    if (!PSF && own) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int r = j + t * M;
            xin[t] = r < nin ? T[r * CG + c] : cplx<R>{R(0), R(0)};
        }
    }
    __syncthreads();   // twiddle table
    const cplx<R> wj = twiddle<R, false>(tt, j << sh2n);
    // image mode: the PSF spectrum at the thread's innermost-stage outputs of a half
    // (8 / R0 items of R0 values), loaded before the middle stages that hide its latency
    // where that measured faster (N <= 2048: 0.101 -> 0.092 ms at 2048^2; at N = 4096 the
    // early loads made the pass 14 % slower), else in the innermost stage
    constexpr int IT = 8 / R0;
    constexpr bool HEXACT = IT * NT == C * (N / R0);
    constexpr bool PREH = LOG2N <= 11;
    R hv[8];
    auto load_h = [&](int p) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int id = threadIdx.x + it * NT;
            if (HEXACT || id < C * (N / R0)) {
                const int cc = id / (N / R0), gq = id - cc * (N / R0);
#pragma unroll
                for (int t = 0; t < R0; ++t) hv[it * R0 + t] = H[(p * N + dit_inv<LOG2N>(gq * R0 + t)) * CG + cc];
            }
        }
    };
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        // forward N-point DFT of the even (p = 0) or odd (p = 1) half by decimation in
        // frequency: the first stage from the inputs, X[k] ends at the DIT position of k
        if (own) {
            cplx<R> v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int r = j + t * M;
                cplx<R> x;
                if (PSF) {
                    const cplx<R> lo = T[r * CG + c], hi = T[(r + N) * CG + c];
                    x = p == 0 ? lo + hi : lo - hi;
                } else {
                    x = xin[t];
                }
                v[t] = p == 0 ? x : x * (wj * root16<R>(t));   // w^r = w^j exp(-2 pi i t / 16)
            }
            dft_small<R, false, 8>(v);
            stage_twiddles<R, false, 8>(v, tt, (j * (N / (8 * M))) << shn);
            cplx<R> *vb = buf + c * ld + LD::pad(j);
#pragma unroll
            for (int t = 0; t < 8; ++t) vb[LD::pad(t * M)] = v[t];
        }
        if (!PSF && PREH) load_h(p);
        __syncthreads();
        {
            int m = M;
#pragma unroll
            for (int st = S - 2; st >= 1; --st) {   // middle stages, radix 8
                m /= 8;
                dif_stage<R, false, 8, LOG2N, NT>(buf, C, ld, m, tt, shn);
                __syncthreads();
            }
        }
        // innermost stage (span 1) of the forward transform, the product with the PSF
        // spectrum and the innermost stage of the inverse, in registers
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int id = threadIdx.x + it * NT;
            if (!HEXACT && id >= C * (N / R0)) continue;
            const int cc = id / (N / R0), gq = id - cc * (N / R0);
            // (without the early loads: this item's spectrum values are loaded first, then
            // the LDS reads and the DFT cover part of their latency)
            R hl[R0];
            if (!PSF && !PREH) {
#pragma unroll
                for (int t = 0; t < R0; ++t) hl[t] = H[(p * N + dit_inv<LOG2N>(gq * R0 + t)) * CG + cc];
            }
            cplx<R> *vb = buf + cc * ld + LD::pad(gq * R0);
            cplx<R> v[R0];
#pragma unroll
            for (int t = 0; t < R0; ++t) v[t] = vb[LD::pad(t)];
            dft_small<R, false, R0>(v);
#pragma unroll
            for (int t = 0; t < R0; ++t) {
                const int k = dit_inv<LOG2N>(gq * R0 + t);
                if (PSF) H[(p * N + k) * CG + cc] = v[t].re;
                else v[t] = v[t] * (PREH ? hv[it * R0 + t] : hl[t]);
            }
            if (!PSF) {
                dft_small<R, true, R0>(v);
#pragma unroll
                for (int t = 0; t < R0; ++t) vb[LD::pad(t)] = v[t];
            }
        }
        __syncthreads();
        if (PSF) continue;
        {
            int m = R0;
#pragma unroll
            for (int st = 1; st <= S - 2; ++st) {   // middle stages of the inverse (DIT)
                dit_stage<R, true, 8, LOG2N, NT>(buf, C, ld, m, tt, shn);
                m *= 8;
                __syncthreads();
            }
        }
        // outermost stage of the inverse, outputs y[j + t M] in registers
        if (own) {
            const cplx<R> *vb = buf + c * ld + LD::pad(j);
            cplx<R> v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = vb[LD::pad(t * M)];
            stage_twiddles<R, true, 8>(v, tt, j << shn);
            dft_small<R, true, 8>(v);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (p == 0) ev[t] = v[t];
                else if (j + t * M < a.nx)   // the crop: rows 0 .. nx - 1
                    Y[(j + t * M) * CG + c] = ev[t] + v[t] * conj(wj * root16<R>(t));
            }
        }
        __syncthreads();
    }
}

// columns per block of the column pass: the most (up to 8) whose C x nx block
// spans at most 512 threads x 8 values (one radix-8 butterfly per thread and
// stage; the even half's outputs stay in registers) and fits the LDS
template <typename R, int LG> constexpr int conv_cgc() {
    constexpr int N = 1 << LG;
    constexpr int budget = (int)(16384 / sizeof(R));   // values of a C x nx block
    constexpr int C = budget / N >= 8 ? 8 : (budget / N >= 1 ? budget / N : 1);
    static_assert(ConvCols<R, LG, C>::lds <= kMaxLdsBytes, "column group exceeds the LDS");
    return C;
}
// layout group width: the column pass's columns per block, at least 32 bytes of a
// row (the row passes store and load 64 contiguous bytes of each row pair; the
// CG / C column-pass blocks of a group share its lines in the L2 of one XCD, and
// more of them per group lose to L2 misses: measured best at 32 bytes)
template <typename R, int LG> constexpr int conv_layout_cg() {
    return conv_cgc<R, LG>() < 32 / (int)sizeof(cplx<R>) ? 32 / (int)sizeof(cplx<R>) : conv_cgc<R, LG>();
}
int conv_group_cols(bool dbl, int nx) {
    int C = 1;
    (void)dispatch_int<4, 12>(__builtin_ctz(nx), [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        C = dbl ? conv_layout_cg<double, LG>() : conv_layout_cg<float, LG>();
        return hipSuccess;
    });
    return C;
}

// S3: inverse row DFT (length 2ny) of the Hermitian half spectrum, real part,
// cropped to ny, scaled by 1 / (4 nx ny), with fused epilogues.
// Inverse of s1's pairing: rows 2c and 2c + 1 have Hermitian half spectra X_a,
// X_b; Z = X_a + i X_b transforms to row a in the real part and row b in the
// imaginary part.  C vectors (2C rows) per block.
template <typename R, int LOG2L, int OUT>
__global__ __launch_bounds__(row_threads<LOG2L>(), row_min_waves<LOG2L>()) void s3_kernel(ConvArgs a, R *y, const R *aux, R sigma, int C) {
    constexpr int L = 1 << LOG2L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *const twl = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf = twl + kTwEntries + row_tw_se<R, LOG2L>();
    const TwTab<R> tt = tw_fill<R, row_threads<LOG2L>(), LOG2L, row_tw_se<R, LOG2L>()>(
        twl, reinterpret_cast<const cplx<R> *>(a.tw), a.log2_lmax);
    __shared__ double red[row_threads<LOG2L>() / 64];
    const int ld = Lds<R, LOG2L>::ld;
    const int nx = a.nx, ny = a.ny;
    const int ngrp = nx / (2 * C);
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int ig = lb % ngrp;
    const int b = lb / ngrp;
    const cplx<R> *t1 = reinterpret_cast<const cplx<R> *>(a.t1c) + (size_t)b * a.lx * a.ldh + conv_out_off(a);
    const int lgc = __builtin_ctz(a.cgc), cmask = a.cgc - 1;
    const R scale = R(1) / ((R)a.lx * (R)a.ly);
    double part = 0.0;
    struct RawS {
        cplx<R> xa, xb;
    };
    constexpr bool READ_AUX = OUT == CONV_OUT_SUB || OUT == CONV_OUT_CG || OUT == CONV_OUT_DOT;
    // eight inputs per thread in flight where that fits the register budget (up to 8192 points)
    row_fft<R, true, LOG2L, row_threads<LOG2L>(), true, fuse_first8<LOG2L>(), (LOG2L <= 13 ? 8 : 0)>(
        buf, C, ld, tt, a.log2_lmax - LOG2L,
        [&](int c, int k) {
            // group-major load of rows i, i + 1 at frequency kk (Hermitian: k > ny reads L - k)
            const int kk = k <= L / 2 ? k : L - k;
            const size_t o = (((size_t)(kk >> lgc) * nx + ig * 2 * C + 2 * c) << lgc) + (kk & cmask);
            return RawS{t1[o], t1[o + a.cgc]};
        },
        [&](int, int k, const RawS &raw) -> cplx<R> {
            const cplx<R> xa = k > L / 2 ? conj(raw.xa) : raw.xa, xb = k > L / 2 ? conj(raw.xb) : raw.xb;
            return cplx<R>{xa.re - xb.im, xa.im + xb.re};
        },
        [&](int c, int j) -> cplx<R> {   // the auxiliary image at the two output pixels
            cplx<R> p{R(0), R(0)};
            if (READ_AUX && j < ny) {
                const size_t pix = ((size_t)b * nx + ig * 2 * C + 2 * c) * ny + j;
                p = cplx<R>{aux[pix], aux[pix + ny]};
            }
            return p;
        },
        [&](int c, int j, const cplx<R> &z, const cplx<R> &p) {
            if (j >= ny) return;
#pragma unroll
            for (int h = 0; h < 2; ++h) {   // rows 2c (real part) and 2c + 1 (imaginary part)
                const size_t pix = ((size_t)b * nx + ig * 2 * C + 2 * c + h) * ny + j;
                const R pv = h ? p.im : p.re;
                R v = (h ? z.im : z.re) * scale;
                if (OUT == CONV_OUT_SUB) v -= pv;
                if (OUT == CONV_OUT_CG) {
                    v += sigma * pv;
                    part += (double)pv * (double)v;
                }
                if (OUT == CONV_OUT_NORM) part += (double)v * (double)v;
                if (OUT == CONV_OUT_DOT) part += (double)pv * (double)v;
                y[pix] = v;
            }
        });
    if (OUT == CONV_OUT_CG || OUT == CONV_OUT_NORM || OUT == CONV_OUT_DOT) {
        const double t = block_sum<row_threads<LOG2L>()>(part, red);
        if (threadIdx.x == 0) a.partials[(size_t)b * a.max_partials + ig] = t;
    }
}

template <typename R>
static hipError_t conv_columns(const ConvArgs &a, int psf, hipStream_t s) {
    return dispatch_int<4, 12>(__builtin_ctz(a.lx) - 1, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        constexpr int CG = conv_layout_cg<R, LG>();
        constexpr int CB = conv_cgc<R, LG>();   // columns per block
        using K = ConvCols<R, LG, CB>;
        if (a.cgc != CG) return hipErrorInvalidValue;
        const int G = (a.ly / 2 + CG) / CG;
        const int nb = ((a.n_band * G + 7) / 8) * 8 * (CG / CB);
        if (psf) PFB_LAUNCH_NT((conv_cols_kernel<R, LG, CB, CG, true>), nb, K::NT, K::lds, s, a);
        else PFB_LAUNCH_NT((conv_cols_kernel<R, LG, CB, CG, false>), nb, K::NT, K::lds, s, a);
        return hipSuccess;
    });
}

// row pairs per block of the row passes: at most cmax, and a power of two that
// divides the nx / 2 pairs of the image
static int conv_row_pairs(int cmax, int nx) {
    int C = 1;
    while (2 * C <= cmax && (nx / 2) % (2 * C) == 0) C *= 2;
    return C;
}

template <typename R>
static hipError_t psf_conv_t(const ConvArgs &a, const void *x, void *aux_in, void *y, const void *aux_out,
                             double sigma, int in_mode, int out_mode, hipStream_t s) {
    const int lg = __builtin_ctz(a.ly);
    hipError_t e = dispatch_int<5, 14>(lg, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        const int C = conv_row_pairs(rows_per_block<R, LG>(), a.nx);   // vectors = row pairs
        const size_t lds = row_lds<R, LG>(C);
        const int nb = a.n_band * (a.nx / (2 * C));
        const R *xr = reinterpret_cast<const R *>(x);
        R *ap = reinterpret_cast<R *>(aux_in);
        if (in_mode == CONV_IN_X) PFB_LAUNCH_NT((s1_kernel<R, LG, CONV_IN_X>), nb, row_threads<LG>(), lds, s, a, xr, ap, a.nx, C, 0);
        else if (in_mode == CONV_IN_CG_P) PFB_LAUNCH_NT((s1_kernel<R, LG, CONV_IN_CG_P>), nb, row_threads<LG>(), lds, s, a, xr, ap, a.nx, C, 0);
        else PFB_LAUNCH_NT((s1_kernel<R, LG, CONV_IN_SCALED>), nb, row_threads<LG>(), lds, s, a, xr, ap, a.nx, C, 0);
        return hipSuccess;
    });
    if (e != hipSuccess) return e;
    e = conv_columns<R>(a, 0, s);
    if (e != hipSuccess) return e;
    return dispatch_int<5, 14>(lg, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        const int C = conv_row_pairs(rows_per_block<R, LG>(), a.nx);   // vectors = row pairs
        const size_t lds = row_lds<R, LG>(C);
        const int nb = a.n_band * (a.nx / (2 * C));
        R *yr = reinterpret_cast<R *>(y);
        const R *ax = reinterpret_cast<const R *>(aux_out);
        const R sg = (R)sigma;
        switch (out_mode) {
            case CONV_OUT_Y: PFB_LAUNCH_NT((s3_kernel<R, LG, CONV_OUT_Y>), nb, row_threads<LG>(), lds, s, a, yr, ax, sg, C); break;
            case CONV_OUT_SUB: PFB_LAUNCH_NT((s3_kernel<R, LG, CONV_OUT_SUB>), nb, row_threads<LG>(), lds, s, a, yr, ax, sg, C); break;
            case CONV_OUT_CG: PFB_LAUNCH_NT((s3_kernel<R, LG, CONV_OUT_CG>), nb, row_threads<LG>(), lds, s, a, yr, ax, sg, C); break;
            case CONV_OUT_NORM: PFB_LAUNCH_NT((s3_kernel<R, LG, CONV_OUT_NORM>), nb, row_threads<LG>(), lds, s, a, yr, ax, sg, C); break;
            default: PFB_LAUNCH_NT((s3_kernel<R, LG, CONV_OUT_DOT>), nb, row_threads<LG>(), lds, s, a, yr, ax, sg, C); break;
        }
        return hipSuccess;
    });
}

hipError_t launch_psf_conv(bool dbl, const ConvArgs &a, const void *x, void *aux_in, void *y, const void *aux_out,
                           double sigma, int in_mode, int out_mode, hipStream_t s) {
    return dbl ? psf_conv_t<double>(a, x, aux_in, y, aux_out, sigma, in_mode, out_mode, s)
               : psf_conv_t<float>(a, x, aux_in, y, aux_out, sigma, in_mode, out_mode, s);
}

int conv_partials_per_band(bool dbl, const ConvArgs &a) {
    // S3 writes one partial per block of 2C rows; C depends on the row length
    const int lg = __builtin_ctz(a.ly);
    int C = 1;
    (void)dispatch_int<5, 14>(lg, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        C = dbl ? rows_per_block<double, LG>() : rows_per_block<float, LG>();
        return hipSuccess;
    });
    return a.nx / (2 * conv_row_pairs(C, a.nx));
}

template <typename R>
static hipError_t psfhat_t(const ConvArgs &a, const void *psf_img, hipStream_t s) {
    const int lg = __builtin_ctz(a.ly);
    hipError_t e = dispatch_int<5, 14>(lg, [&](auto Lc) -> hipError_t {
        constexpr int LG = decltype(Lc)::value;
        const int C = std::min(rows_per_block<R, LG>(), a.lx / 2);      // vectors = row pairs of lx rows
        const size_t lds = row_lds<R, LG>(C);
        const int nb = a.n_band * (a.lx / (2 * C));
        PFB_LAUNCH_NT((s1_kernel<R, LG, CONV_IN_X>), nb, row_threads<LG>(), lds, s, a, reinterpret_cast<const R *>(psf_img),
                   (R *)nullptr, a.lx, C, 1);
        return hipSuccess;
    });
    if (e != hipSuccess) return e;
    return conv_columns<R>(a, 1, s);
}
hipError_t launch_psfhat(bool dbl, const ConvArgs &a, const void *psf_img, hipStream_t s) {
    return dbl ? psfhat_t<double>(a, psf_img, s) : psfhat_t<float>(a, psf_img, s);
}

// ---------------------------------------------------------------------------
// vector kernels and device-side scalar reductions
// ---------------------------------------------------------------------------
constexpr int kVecPerThread = 8;

int vec_partials_per_band(int64_t P) {
    const int64_t per = (int64_t)kThreads * kVecPerThread;
    int64_t n = (P + per - 1) / per;
    return (int)std::min<int64_t>(n, 4096);
}

template <typename R, int OP>
__global__ __launch_bounds__(kThreads) void vec_kernel(int64_t P, int nblk, double *partials, int max_partials,
                                                       const double *scal, R *x, R *y, R *r, R *p, const R *ap,
                                                       R gamma, R lam) {
    __shared__ double red[kThreads / 64];
    const int b = blockIdx.x / nblk;
    const int kb = blockIdx.x - b * nblk;
    const size_t off = (size_t)b * P;
    const double *sc = scal + b * 8;
    double part = 0.0;
    const R alpha = (OP == VEC_CG_UPDATE) ? (R)sc[S_ALPHA] : R(0);
    const R scale = (OP == VEC_SCALE_COPY) ? (R)sc[S_SCALE] : R(1);
    for (int64_t k = (int64_t)kb * kThreads + threadIdx.x; k < P; k += (int64_t)nblk * kThreads) {
        const size_t e = off + k;
        if (OP == VEC_CG_INIT) {
            const R g = x[e];
            y[e] = R(0);
            r[e] = g;
            p[e] = R(0);
            part += (double)g * (double)g;
        } else if (OP == VEC_CG_UPDATE) {
            y[e] += alpha * p[e];
            const R rn = r[e] - alpha * ap[e];
            r[e] = rn;
            part += (double)rn * (double)rn;
        } else if (OP == VEC_SCALE_COPY) {
            y[e] = x[e] * scale;
        } else if (OP == VEC_DOT) {
            part += (double)x[e] * (double)y[e];
        } else if (OP == VEC_FB_PROX) {
            const R v = x[e] - gamma * y[e] - gamma * lam;
            x[e] = v > R(0) ? v : R(0);
        } else if (OP == VEC_NORM) {
            part += (double)x[e] * (double)x[e];
        }
    }
    if (OP == VEC_CG_INIT || OP == VEC_CG_UPDATE || OP == VEC_DOT || OP == VEC_NORM) {
        const double t = block_sum(part, red);
        if (threadIdx.x == 0) partials[(size_t)b * max_partials + kb] = t;
    }
}

hipError_t launch_vec(bool dbl, int op, int n_band, int64_t P, double *partials, int max_partials,
                      const double *scal, void *x, void *y, void *r, void *p, const void *ap, double gamma,
                      double lam, hipStream_t s) {
    const int nblk = vec_partials_per_band(P);
    const int nb = n_band * nblk;
#define VEC_CASE(T, OPV)                                                                                    \
    case OPV:                                                                                               \
        PFB_LAUNCH((vec_kernel<T, OPV>), nb, 0, s, P, nblk, partials, max_partials, scal, (T *)x, (T *)y, \
                   (T *)r, (T *)p, (const T *)ap, (T)gamma, (T)lam);                                       \
        break;
    if (dbl) {
        switch (op) {
            VEC_CASE(double, VEC_CG_INIT)
            VEC_CASE(double, VEC_CG_UPDATE)
            VEC_CASE(double, VEC_SCALE_COPY)
            VEC_CASE(double, VEC_DOT)
            VEC_CASE(double, VEC_FB_PROX)
            VEC_CASE(double, VEC_NORM)
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (op) {
            VEC_CASE(float, VEC_CG_INIT)
            VEC_CASE(float, VEC_CG_UPDATE)
            VEC_CASE(float, VEC_SCALE_COPY)
            VEC_CASE(float, VEC_DOT)
            VEC_CASE(float, VEC_FB_PROX)
            VEC_CASE(float, VEC_NORM)
            default: return hipErrorInvalidValue;
        }
    }
#undef VEC_CASE
    return hipSuccess;
}

// One workgroup per band sums that band's partials (fixed order) and updates
// the band's scalars.
__global__ __launch_bounds__(kThreads) void reduce_kernel(int op, const double *partials, int n_part,
                                                          int max_partials, double *scal) {
    __shared__ double red[kThreads / 64];
    const int b = blockIdx.x;
    double v = 0.0;
    for (int k = threadIdx.x; k < n_part; k += kThreads) v += partials[(size_t)b * max_partials + k];
    const double t = block_sum(v, red);
    if (threadIdx.x != 0) return;
    double *sc = scal + b * 8;
    switch (op) {
        case RED_SET_RR:
            sc[S_RR] = t;
            sc[S_RR0] = t;
            sc[S_BETA] = 0.0;
            break;
        case RED_ALPHA:
            sc[S_PAP] = t;
            sc[S_ALPHA] = (t > 0.0 && sc[S_RR] > 0.0) ? sc[S_RR] / t : 0.0;
            break;
        case RED_BETA:
            sc[S_BETA] = sc[S_RR] > 0.0 ? t / sc[S_RR] : 0.0;
            sc[S_RR] = t;
            break;
        case RED_INV_SQRT:
            sc[S_SCALE] = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
            break;
        case RED_LAMBDA:
            sc[S_LAMBDA] = t;
            break;
        default:
            sc[S_TMP] = t;
            break;
    }
}

hipError_t launch_reduce(int op, int n_band, const double *partials, int n_part, int max_partials, double *scal,
                         hipStream_t s) {
    PFB_LAUNCH(reduce_kernel, n_band, 0, s, op, partials, n_part, max_partials, scal);
    return hipSuccess;
}

__global__ void copy_scalar_kernel(int n_band, const double *scal, int slot, double *dst) {
    const int b = threadIdx.x;
    if (b < n_band) dst[b] = scal[b * 8 + slot];
}
hipError_t launch_copy_scalar(int n_band, const double *scal, int slot, double *dst, hipStream_t s) {
    for (int b0 = 0; b0 < n_band; b0 += kThreads) {
        PFB_LAUNCH(copy_scalar_kernel, 1, 0, s, n_band - b0, scal + (size_t)b0 * 8, slot, dst + b0);
    }
    return hipSuccess;
}


// ---------------------------------------------------------------------------
// backward step (eq. 7 with the regulariser of eq. 9): wavelet dictionary and
// primal-dual updates
// ---------------------------------------------------------------------------
// Taps of one wavelet filter pair in the kernel's precision: low-pass h and
// wavelet g[j] = (-1)^j h[2N-1-j].
template <typename R> struct WaveletTaps {
    R h[kMaxWaveletTaps], g[kMaxWaveletTaps];
};
static int64_t wave_blocks(int64_t total) {
    int64_t nb = (total + kThreads - 1) / kThreads;
    return nb < 1 ? 1 : (nb > 65536 ? 65536 : nb);
}

// One whole 2-D level per launch, in LDS tiles (rows pass, then columns pass,
// the order of the level's definition), so a level reads its block once (plus a
// halo of 2N - 2) and writes it once.  Analysis: a workgroup makes the four
// coefficients (LL, LH, HL, HH) of kWaveTileR x kWaveTileC coefficient positions; LL goes
// to dst_ll (the next level's input, or the coefficient array after the last
// level), the details to dst_d at the level's quadrant positions.  Synthesis: a
// workgroup makes 2 kWaveTileR x 2 kWaveTileC samples from the LL block (src_ll) and the
// three detail quadrants (src_d), columns pass then rows pass (the adjoint order);
// ACC adds into dst.  Rows `ld` apart, images `img` apart, periodic boundaries.
constexpr int kWaveTileR = 16, kWaveTileC = 32;
template <typename R, int N>
__global__ __launch_bounds__(kThreads) void wavelet_ana2_kernel(const R *src, R *dst_d, R *dst_ll, WaveletTaps<R> f,
                                                                int nr, int nc, int ld, int64_t img) {
    constexpr int TR = kWaveTileR, TC = kWaveTileC;
    constexpr int IR = 2 * TR + 2 * N - 2, IC = 2 * TC + 2 * N - 2;
    __shared__ R xin[IR][IC + 1];
    __shared__ R trow[IR][2 * TC + 1];
    const int hr = nr >> 1, hc = nc >> 1;
    const int kr0 = blockIdx.y * TR, kc0 = blockIdx.x * TC;
    const R *sp = src + (size_t)blockIdx.z * img;
    // the tile wraps round the block only at its far edges (periodic boundaries)
    const bool wrap = 2 * kr0 + IR > nr || 2 * kc0 + IC > nc;
    for (int id = threadIdx.x; id < IR * IC; id += kThreads) {
        const int r = id / IC, c = id - r * IC;
        int gr = 2 * kr0 + r, gc = 2 * kc0 + c;
        if (wrap) {
            gr %= nr;
            gc %= nc;
        }
        xin[r][c] = sp[(size_t)gr * ld + gc];
    }
    __syncthreads();
    // rows: a thread makes KB consecutive (low, high) pairs from one window of
    // 2N + 2KB - 2 samples held in registers
    constexpr int KB = 4, WIN = 2 * N + 2 * KB - 2;
    for (int id = threadIdx.x; id < IR * (TC / KB); id += kThreads) {
        const int r = id / (TC / KB), k0 = (id - r * (TC / KB)) * KB;
        R x[WIN];
#pragma unroll
        for (int t = 0; t < WIN; ++t) x[t] = xin[r][2 * k0 + t];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            R lo = R(0), hi = R(0);
#pragma unroll
            for (int j = 0; j < 2 * N; ++j) {
                lo += f.h[j] * x[2 * u + j];
                hi += f.g[j] * x[2 * u + j];
            }
            trow[r][k0 + u] = lo;
            trow[r][TC + k0 + u] = hi;
        }
    }
    __syncthreads();
    R *dd = dst_d + (size_t)blockIdx.z * img;
    R *dl = dst_ll + (size_t)blockIdx.z * img;
    // columns: KB consecutive coefficient rows per thread, as above
    for (int id = threadIdx.x; id < (TR / KB) * 2 * TC; id += kThreads) {
        const int kb = id / (2 * TC), c = id - kb * (2 * TC);
        const int kr0b = kb * KB;
        const bool chi = c >= TC;
        const int kc = chi ? c - TC : c;
        if (kc0 + kc >= hc) continue;
        R t[WIN];
#pragma unroll
        for (int v = 0; v < WIN; ++v) t[v] = trow[2 * kr0b + v][c];
        const int col = (chi ? hc : 0) + kc0 + kc;
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int kr = kr0b + u;
            if (kr0 + kr >= hr) break;
            R lo = R(0), hi = R(0);
#pragma unroll
            for (int j = 0; j < 2 * N; ++j) {
                lo += f.h[j] * t[2 * u + j];
                hi += f.g[j] * t[2 * u + j];
            }
            if (chi) dd[(size_t)(kr0 + kr) * ld + col] = lo;
            else dl[(size_t)(kr0 + kr) * ld + col] = lo;
            dd[(size_t)(hr + kr0 + kr) * ld + col] = hi;
        }
    }
}

template <typename R, int N, bool ACC>
__global__ __launch_bounds__(kThreads) void wavelet_syn2_kernel(const R *src_ll, const R *src_d, R *dst,
                                                                WaveletTaps<R> f, int nr, int nc, int ld, int64_t img) {
    constexpr int TR = kWaveTileR, TC = kWaveTileC;
    constexpr int YR = TR + N - 1, YC = TC + N - 1;   // coefficient rows / columns per half
    __shared__ R yin[2 * YR][2 * YC + 1];
    __shared__ R tcol[2 * TR][2 * YC + 1];
    const int hr = nr >> 1, hc = nc >> 1;
    const int kr0 = blockIdx.y * TR, kc0 = blockIdx.x * TC;
    const R *sl = src_ll + (size_t)blockIdx.z * img;
    const R *sd = src_d + (size_t)blockIdx.z * img;
    // the coefficient window wraps only at the block's edges (periodic boundaries)
    const bool wrap = kr0 < N - 1 || kc0 < N - 1 || kr0 + YR - (N - 1) > hr || kc0 + YC - (N - 1) > hc;
    for (int id = threadIdx.x; id < 4 * YR * YC; id += kThreads) {
        const int a = id / (2 * YC), b = id - a * (2 * YC);
        const bool rhi = a >= YR, chi = b >= YC;
        int pr = (rhi ? a - YR : a) + kr0 - (N - 1), pc = (chi ? b - YC : b) + kc0 - (N - 1);
        if (wrap) {
            while (pr < 0) pr += hr;
            while (pc < 0) pc += hc;
            pr %= hr;
            pc %= hc;
        }
        const size_t off = (size_t)((rhi ? hr : 0) + pr) * ld + (chi ? hc : 0) + pc;
        yin[a][b] = (!rhi && !chi) ? sl[off] : sd[off];
    }
    __syncthreads();
    // columns: sample rows 2p + e of the tile from coefficient rows p - i, i < N;
    // a thread makes PB consecutive p (both e) from PB + N - 1 low and high rows
    constexpr int PB = 4, PW = PB + N - 1;
    for (int id = threadIdx.x; id < (TR / PB) * 2 * YC; id += kThreads) {
        const int pb = id / (2 * YC), b = id - pb * (2 * YC);
        const int p0 = pb * PB;
        R lo[PW], hi[PW];
#pragma unroll
        for (int t = 0; t < PW; ++t) {
            lo[t] = yin[p0 + t][b];
            hi[t] = yin[YR + p0 + t][b];
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                R acc = R(0);
#pragma unroll
                for (int i = 0; i < N; ++i) acc += f.h[2 * i + e] * lo[u + N - 1 - i] + f.g[2 * i + e] * hi[u + N - 1 - i];
                tcol[2 * (p0 + u) + e][b] = acc;
            }
        }
    }
    __syncthreads();
    R *dp = dst + (size_t)blockIdx.z * img;
    // rows: PB consecutive q (both e) per thread, as above
    for (int id = threadIdx.x; id < 2 * TR * (TC / PB); id += kThreads) {
        const int mr = id / (TC / PB), q0 = (id - mr * (TC / PB)) * PB;
        if (kr0 + (mr >> 1) >= hr) continue;
        R lo[PW], hi[PW];
#pragma unroll
        for (int t = 0; t < PW; ++t) {
            lo[t] = tcol[mr][q0 + t];
            hi[t] = tcol[mr][YC + q0 + t];
        }
        R *orow = dp + (size_t)(2 * kr0 + mr) * ld + 2 * kc0;
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            if (kc0 + q0 + u >= hc) break;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                R acc = R(0);
#pragma unroll
                for (int i = 0; i < N; ++i) acc += f.h[2 * i + e] * lo[u + N - 1 - i] + f.g[2 * i + e] * hi[u + N - 1 - i];
                R *o = orow + 2 * (q0 + u) + e;
                if (ACC) *o += acc;
                else *o = acc;
            }
        }
    }
}

template <typename R>
static WaveletTaps<R> make_taps(const WaveletFilter &f) {
    WaveletTaps<R> t{};
    const int L = f.len;
    for (int j = 0; j < L; ++j) {
        t.h[j] = (R)f.h[j];
        t.g[j] = (R)((j & 1) ? -f.h[L - 1 - j] : f.h[L - 1 - j]);
    }
    return t;
}

template <typename R>
static hipError_t wavelet_level_t(bool inv, bool acc, const void *a_src, const void *b_src, void *a_dst, void *b_dst,
                                  const WaveletFilter &f, int nr, int nc, int ld, int64_t img, int n_img,
                                  hipStream_t s) {
    const int L = f.len;
    if (L < 2 || L > kMaxWaveletTaps || (L & 1) || nr < 2 || nc < 2 || (nr & 1) || (nc & 1) || n_img > 65535)
        return hipErrorInvalidValue;
    const WaveletTaps<R> t = make_taps<R>(f);
    const dim3 grid((nc / 2 + kWaveTileC - 1) / kWaveTileC, (nr / 2 + kWaveTileR - 1) / kWaveTileR, n_img);
    if (grid.y > 65535) return hipErrorInvalidValue;
    return dispatch_int<1, 6>(L / 2, [&](auto Nc) -> hipError_t {
        constexpr int N = decltype(Nc)::value;
        if (!inv) {
            PFB_LAUNCH((wavelet_ana2_kernel<R, N>), grid, 0, s, (const R *)a_src, (R *)a_dst, (R *)b_dst, t, nr, nc,
                       ld, img);
        } else if (acc) {
            PFB_LAUNCH((wavelet_syn2_kernel<R, N, true>), grid, 0, s, (const R *)a_src, (const R *)b_src, (R *)a_dst,
                       t, nr, nc, ld, img);
        } else {
            PFB_LAUNCH((wavelet_syn2_kernel<R, N, false>), grid, 0, s, (const R *)a_src, (const R *)b_src, (R *)a_dst,
                       t, nr, nc, ld, img);
        }
        return hipSuccess;
    });
}

hipError_t launch_wavelet_analysis_level(bool dbl, const void *src, void *dst_detail, void *dst_ll,
                                         const WaveletFilter &f, int nr, int nc, int ld, int64_t img, int n_img,
                                         hipStream_t s) {
    if (dbl) return wavelet_level_t<double>(false, false, src, nullptr, dst_detail, dst_ll, f, nr, nc, ld, img, n_img, s);
    return wavelet_level_t<float>(false, false, src, nullptr, dst_detail, dst_ll, f, nr, nc, ld, img, n_img, s);
}

hipError_t launch_wavelet_synthesis_level(bool dbl, bool acc, const void *src_ll, const void *src_detail, void *dst,
                                          const WaveletFilter &f, int nr, int nc, int ld, int64_t img, int n_img,
                                          hipStream_t s) {
    if (dbl) return wavelet_level_t<double>(true, acc, src_ll, src_detail, dst, nullptr, f, nr, nc, ld, img, n_img, s);
    return wavelet_level_t<float>(true, acc, src_ll, src_detail, dst, nullptr, f, nr, nc, ld, img, n_img, s);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void wave_copy_kernel(const R *src, R *dst, int64_t n, R scale) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[i] * scale;
}
template <typename R>
__global__ __launch_bounds__(kThreads) void wave_axpy_kernel(const R *x, const R *y, R *z, int64_t n, R a) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        z[i] = x[i] + a * y[i];
}
hipError_t launch_wave_axpy(bool dbl, const void *x, const void *y, void *z, int64_t n, double a, hipStream_t s) {
    const int64_t nb = wave_blocks(n);
    if (dbl)
        PFB_LAUNCH(wave_axpy_kernel<double>, nb, 0, s, (const double *)x, (const double *)y, (double *)z, n, a);
    else
        PFB_LAUNCH(wave_axpy_kernel<float>, nb, 0, s, (const float *)x, (const float *)y, (float *)z, n, (float)a);
    return hipSuccess;
}

hipError_t launch_wave_copy(bool dbl, const void *src, void *dst, int64_t n, double scale, hipStream_t s) {
    const int64_t nb = wave_blocks(n);
    if (dbl)
        PFB_LAUNCH(wave_copy_kernel<double>, nb, 0, s, (const double *)src, (double *)dst, n, scale);
    else
        PFB_LAUNCH(wave_copy_kernel<float>, nb, 0, s, (const float *)src, (float *)dst, n, (float)scale);
    return hipSuccess;
}

// Primal update of the primal-dual iteration, per pixel:
//   x~ = max(x - tau ((c + sigma_u d) / gamma + psi_scale * s), 0),   d = x - z, c = I^psf * d
//   u  = 2 x~ - x;  x = x~;  d = x~ - z
// INIT (before the first iteration): x = max(z, 0) unless warm, d = x - z.
template <typename R, bool INIT>
__global__ __launch_bounds__(kThreads) void pd_primal_kernel(const R *z, R *x, R *d, const R *c, const R *sv, R *u,
                                                             int64_t n, R tau, R inv_gamma, R sigma_u, R psi_scale,
                                                             int warm) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        if (INIT) {
            const R xi = warm ? x[i] : max(z[i], R(0));
            x[i] = xi;
            d[i] = xi - z[i];
        } else {
            const R xi = x[i], di = d[i];
            const R grad = (c[i] + sigma_u * di) * inv_gamma;
            const R xt = max(xi - tau * (grad + psi_scale * sv[i]), R(0));
            u[i] = R(2) * xt - xi;
            x[i] = xt;
            d[i] = xt - z[i];
        }
    }
}

// Dual update per (basis, coefficient): t_b = v_b + sigma_d psi_scale a_b over the
// bands b, v = t min(1, lam / ||t||_2); basis 0 reads the image u (Dirac), basis
// k >= 1 its analysis coefficients.  ZERO: v = 0.
template <typename R, bool ZERO>
__global__ __launch_bounds__(kThreads) void pd_dual_kernel(R *v, const R *u, const R *coef, int nbasis, int n_band,
                                                           int64_t P, R sigma_d, R psi_scale, R lam) {
    const int64_t total = (int64_t)nbasis * P;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int k = (int)(id / P);
        const int64_t p = id - (int64_t)k * P;
        R *vk = v + (size_t)k * n_band * P + p;
        if (ZERO) {
            for (int b = 0; b < n_band; ++b) vk[(size_t)b * P] = R(0);
            continue;
        }
        const R *ak = k == 0 ? u + p : coef + (size_t)(k - 1) * n_band * P + p;
        double nrm2 = 0.0;
        for (int b = 0; b < n_band; ++b) {
            const R t = vk[(size_t)b * P] + sigma_d * psi_scale * ak[(size_t)b * P];
            nrm2 += (double)t * (double)t;
        }
        const double nrm = sqrt(nrm2);
        const R sc = nrm > (double)lam ? (R)((double)lam / nrm) : R(1);
        for (int b = 0; b < n_band; ++b) {
            const R t = vk[(size_t)b * P] + sigma_d * psi_scale * ak[(size_t)b * P];
            vk[(size_t)b * P] = t * sc;
        }
    }
}

hipError_t launch_pd_primal(bool dbl, bool init, const void *z, void *x, void *d, const void *c, const void *sv,
                            void *u, int64_t n, double tau, double gamma, double sigma_u, double psi_scale, int warm,
                            hipStream_t s) {
    const int64_t nb = wave_blocks(n);
#define PDP(T)                                                                                                    \
    if (init)                                                                                                     \
        PFB_LAUNCH((pd_primal_kernel<T, true>), nb, 0, s, (const T *)z, (T *)x, (T *)d, (const T *)c,           \
                   (const T *)sv, (T *)u, n, (T)tau, (T)(1.0 / gamma), (T)sigma_u, (T)psi_scale, warm);          \
    else                                                                                                          \
        PFB_LAUNCH((pd_primal_kernel<T, false>), nb, 0, s, (const T *)z, (T *)x, (T *)d, (const T *)c,          \
                   (const T *)sv, (T *)u, n, (T)tau, (T)(1.0 / gamma), (T)sigma_u, (T)psi_scale, warm);
    if (dbl) {
        PDP(double)
    } else {
        PDP(float)
    }
#undef PDP
    return hipSuccess;
}

hipError_t launch_pd_dual(bool dbl, bool zero, void *v, const void *u, const void *coef, int nbasis, int n_band,
                          int64_t P, double sigma_d, double psi_scale, double lam, hipStream_t s) {
    const int64_t nb = wave_blocks((int64_t)nbasis * P);
#define PDD(T)                                                                                                  \
    if (zero)                                                                                                   \
        PFB_LAUNCH((pd_dual_kernel<T, true>), nb, 0, s, (T *)v, (const T *)u, (const T *)coef, nbasis, n_band, \
                   P, (T)sigma_d, (T)psi_scale, (T)lam);                                                        \
    else                                                                                                        \
        PFB_LAUNCH((pd_dual_kernel<T, false>), nb, 0, s, (T *)v, (const T *)u, (const T *)coef, nbasis, n_band,\
                   P, (T)sigma_d, (T)psi_scale, (T)lam);
    if (dbl) {
        PDD(double)
    } else {
        PDD(float)
    }
#undef PDD
    return hipSuccess;
}

}  // namespace pfb
