// Host side of the C ABI: plan creation (validation, w-range analysis,
// bucket counting, work lists, correction and twiddle tables, workspace
// layout) and the operator entry points, which only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "pfb.h"
#include "pfb_kernels.h"

using namespace pfb;

namespace {

thread_local std::string g_last_error = "no error";

pfb_status fail(pfb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_OK(expr)                                                                     \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return fail(PFB_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));       \
    } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
// smallest power of two >= v (v >= 1)
int next_pow2(int64_t v) {
    int p = 1;
    while (p < v) p *= 2;
    return p;
}
int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

// ---- Fourier transform of the ES kernel --------------------------------------
// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
}

// psi_hat(xi) = int phi(x) exp(2 pi i x xi) dx over |x| < W/2, with x = (W/2) sin(theta)
// removing the square-root edge of the ES kernel so the quadrature converges fast.
struct PsiHat {
    int W;
    double beta;
    std::vector<double> th, wt;
    PsiHat(int W_, double beta_) : W(W_), beta(beta_) {
        std::vector<double> x, w;
        gauss_legendre(160, x, w);
        th.resize(x.size());
        wt.resize(x.size());
        for (size_t k = 0; k < x.size(); ++k) {
            th[k] = 0.25 * M_PI * (x[k] + 1.0);
            wt[k] = 0.25 * M_PI * w[k];
        }
    }
    double operator()(double xi) const {
        double s = 0.0;
        for (size_t k = 0; k < th.size(); ++k)
            s += wt[k] * std::exp(beta * (std::cos(th[k]) - 1.0)) * std::cos(M_PI * W * xi * std::sin(th[k])) *
                 std::cos(th[k]);
        return W * s;
    }
};

// Chebyshev coefficients of psi_hat in y = 2 (xi / xi_max)^2 - 1.
std::vector<double> psihat_chebyshev(const PsiHat &f, double xi_max, int K, double *max_rel_err) {
    std::vector<double> fk(K), c(K);
    for (int k = 0; k < K; ++k) {
        const double y = std::cos(M_PI * (k + 0.5) / K);
        fk[k] = f(xi_max * std::sqrt(0.5 * (y + 1.0)));
    }
    for (int j = 0; j < K; ++j) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += fk[k] * std::cos(M_PI * j * (k + 0.5) / K);
        c[j] = 2.0 * s / K;
    }
    c[0] *= 0.5;
    double err = 0.0;
    for (int t = 0; t <= 200; ++t) {
        const double xi = xi_max * t / 200.0;
        const double y = 2.0 * (xi / xi_max) * (xi / xi_max) - 1.0;
        double b1 = 0, b2 = 0;
        for (int k = K - 1; k >= 1; --k) {
            const double b0 = c[k] + 2.0 * y * b1 - b2;
            b2 = b1;
            b1 = b0;
        }
        const double v = c[0] + y * b1 - b2;
        const double ref = f(xi);
        err = std::max(err, std::fabs(v - ref) / std::fabs(ref));
    }
    *max_rel_err = err;
    return c;
}

// ---- workspace layout --------------------------------------------------------
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

}  // namespace

// One NUFFT configuration (main w-stacked operator or the flat PSF gridder).
struct GridderHost {
    GeomDev g{};
    std::vector<BandDev> bands;
    std::vector<int64_t> offsets;        // n_band * ntiles * nj0max + 1
    std::vector<int64_t> hoffsets;       // same, over the home-entry list
    int64_t n_home = 0;
    std::vector<GridWork> gwork;
    std::vector<InterpWork> iwork;
    std::vector<int> gband_start, iband_start;  // per band first work item (n_band + 1)
    std::vector<int64_t> sort_items;     // [start, count, band, bucket] of every non-empty bucket
    // per (band, plane, tile): occ = the spread puts non-zero values there; need = the
    // interpolation may read it (occ dilated by one tile, the halo reach)
    std::vector<uint8_t> occ, need;
    std::vector<uint8_t> occ_row, need_row;   // per (band, plane, tile row): any such tile
    // the (band nwmax + plane) ntx + tile row of every set occ_row / need_row flag,
    // band-major, with per-band starts (n_band + 1)
    std::vector<int32_t> occ_list, need_list;
    std::vector<int> occ_list_start, need_list_start;
    bool mfma = false;                   // FP32 w-stacked: matrix-core spread (window sort, phase table)
    int sort_rb = 1, sort_cb = 1;        // sort blocks of base rows x columns
    int64_t n_entries = 0;
    size_t o_sortitems = 0;
    // workspace offsets
    size_t o_bands = 0, o_offsets = 0, o_cursor = 0, o_gwork = 0, o_iwork = 0, o_recs = 0, o_omega = 0;
    size_t o_corr2d = 0, o_corrx = 0, o_corry = 0, o_occ = 0, o_need = 0, o_occ_row = 0, o_need_row = 0;
    size_t o_occ_list = 0, o_need_list = 0;
    bool corr2d = true;
    // device pointers (valid after set_workspace)
    BandDev *d_bands = nullptr;
    int64_t *d_offsets = nullptr;
    unsigned long long *d_cursor = nullptr;
    GridWork *d_gwork = nullptr;
    InterpWork *d_iwork = nullptr;
    void *d_recs = nullptr, *d_omega = nullptr, *d_corr2d = nullptr, *d_corrx = nullptr, *d_corry = nullptr;
    size_t o_phase = 0;
    void *d_phase = nullptr;
    size_t o_hidx = 0, o_hoffsets = 0;
    uint32_t *d_hidx = nullptr;
    int64_t *d_hoffsets = nullptr;
    size_t o_home_pos = 0;           // main gridder: per entry, home-list position of its visibility
    uint32_t *d_home_pos = nullptr;
    const uint8_t *d_occ = nullptr, *d_need = nullptr, *d_occ_row = nullptr, *d_need_row = nullptr;
    const int32_t *d_occ_list = nullptr, *d_need_list = nullptr;
    int64_t keys() const { return (int64_t)g.n_band * g.ntx * g.nty * g.nj0max; }
};

struct pfb_plan {
    pfb_problem prob{};
    pfb_options opt{};
    bool dbl = false;
    size_t rsz = 4;
    std::vector<int32_t> chan_band;
    std::vector<double> freq;
    GridderHost main, psf;
    int64_t n_active = 0, n_flagged = 0;
    double s_min = 0.0, s_max = 0.0;
    int band_batch = 1;
    int conv_cgc = 1;
    int conv_lx = 0, conv_ly = 0;
    int ldh = 0;
    int log2_lmax = 0;
    std::vector<double> cheb;
    double xi_max = 0.25;
    std::vector<double> tw_host;   // interleaved (re, im) float64
    std::vector<float> tw_f32;     // staging copies that outlive asynchronous uploads
    std::vector<int> cb_host;
    int max_partials = 0;
    // workspace
    size_t ws_bytes = 0;
    char *ws = nullptr;
    bool counted = false, ws_ready = false, psf_ready = false;
    size_t o_freq = 0, o_cb = 0, o_cheb = 0, o_tw = 0, o_flagged = 0, o_flagcur = 0;
    size_t o_planes = 0, o_t1 = 0, o_vals = 0, o_psfimg = 0;
    size_t o_t1c = 0, o_psfhat = 0, o_vec = 0, o_partials = 0, o_scal = 0, o_absmax = 0;
    size_t planes_bytes = 0, t_bytes = 0, vec_bytes = 0;
    size_t o_sorttmp = 0;   // scratch for the plan-time sort (aliases the w-plane area when it fits)
    Profiler prof;
    bool prof_on = false;
    void *p(size_t off) const { return ws + off; }
};

namespace {

GeomDev base_geom(const pfb_plan &P, int nx, int ny, bool flat) {
    GeomDev g{};
    g.nx = nx;
    g.ny = ny;
    // oversampled grid: the smallest power of two >= 2 n (sigma = 2 for power-of-two
    // sides, 2 .. 4 otherwise; the ES kernel's error only falls with sigma)
    g.gx = next_pow2(2 * (int64_t)nx);
    g.gy = next_pow2(2 * (int64_t)ny);
    g.T = P.opt.tile;
    g.ntx = g.gx / g.T;
    g.nty = g.gy / g.T;
    g.W = P.opt.support;
    g.n_band = P.prob.n_band;
    g.flat = flat ? 1 : 0;
    g.offx = flat ? 0 : P.prob.offx;   // the flat (PSF) gridder is shift invariant
    g.offy = flat ? 0 : P.prob.offy;
    g.cellx = P.prob.cellx;
    g.celly = P.prob.celly;
    g.beta = 2.30 * g.W;
    return g;
}

// Work lists from the per-(band, tile, base plane) counts.
void build_work(GridderHost &G, const std::vector<unsigned> &counts, const std::vector<unsigned> &hcounts, int chunk) {
    const GeomDev &g = G.g;
    const int ntiles = g.ntx * g.nty;
    const int W = g.flat ? 1 : g.W;
    G.gwork.clear();
    G.iwork.clear();
    G.gband_start.assign(g.n_band + 1, 0);
    G.iband_start.assign(g.n_band + 1, 0);
    std::vector<std::pair<int64_t, GridWork>> gw;
    std::vector<std::pair<int64_t, InterpWork>> iw;
    const size_t nflag = (size_t)g.n_band * g.nwmax * ntiles;
    G.occ.assign(nflag, 0);
    G.need.assign(nflag, 0);
    G.occ_row.assign((size_t)g.n_band * g.nwmax * g.ntx, 0);
    G.need_row.assign((size_t)g.n_band * g.nwmax * g.ntx, 0);
    for (int b = 0; b < g.n_band; ++b) {
        const BandDev &bd = G.bands[b];
        gw.clear();
        iw.clear();
        for (int t = 0; t < ntiles; ++t) {
            const int64_t kb = ((int64_t)b * ntiles + t) * g.nj0max;
            const unsigned *c = counts.data() + kb;
            int64_t tot = 0;
            for (int q = 0; q < bd.nj0; ++q) {
                tot += c[q];
                if (c[q])   // base plane q reaches planes q .. q + W - 1
                    for (int p = q; p < std::min(q + W, bd.nw); ++p) G.occ[((size_t)b * g.nwmax + p) * ntiles + t] = 1;
            }
            // spread items: split the plane range so each item sees <= chunk entries;
            // tiles without entries get none (the row transforms read them as zero)
            const int nw = tot ? bd.nw : 0;
            int p0 = 0;
            while (p0 < nw) {
                int p1 = p0 + 1;
                auto cost = [&](int a0, int a1) {
                    int64_t s = 0;
                    for (int q = std::max(0, a0 - W + 1); q < std::min(a1, bd.nj0); ++q) s += c[q];
                    return s;
                };
                while (p1 < nw && cost(p0, p1 + 1) <= chunk) ++p1;
                gw.push_back({cost(p0, p1) * (int64_t)W + 1, GridWork{b, t, p0, p1}});
                p0 = p1;
            }
            // interpolation items: runs of <= chunk home entries
            const unsigned *hc = hcounts.data() + kb;
            int64_t htot = 0;
            for (int q2 = 0; q2 < bd.nj0; ++q2) htot += hc[q2];
            int64_t e = G.hoffsets[kb];
            const int64_t eend = e + htot;
            int q = 0;
            int64_t qend = G.hoffsets[kb] + hc[0];
            while (e < eend) {
                while (e >= qend) qend += hc[++q];
                const int64_t e1 = std::min(eend, e + chunk);
                int q1 = q;
                int64_t qe = qend;
                while (e1 > qe) qe += hc[++q1];
                iw.push_back({e1 - e, InterpWork{b, t, (int)e, (int)e1, q, q1}});
                e = e1;
            }
        }
        // need: occ of the tile or of one of its 8 neighbours (periodic grid)
        for (int p = 0; p < g.nwmax; ++p) {
            const uint8_t *o = G.occ.data() + ((size_t)b * g.nwmax + p) * ntiles;
            uint8_t *nd = G.need.data() + ((size_t)b * g.nwmax + p) * ntiles;
            for (int tu = 0; tu < g.ntx; ++tu)
                for (int tv = 0; tv < g.nty; ++tv) {
                    if (!o[tu * g.nty + tv]) continue;
                    for (int du = -1; du <= 1; ++du)
                        for (int dv = -1; dv <= 1; ++dv)
                            nd[((tu + du + g.ntx) % g.ntx) * g.nty + (tv + dv + g.nty) % g.nty] = 1;
                }
            uint8_t *orow = G.occ_row.data() + ((size_t)b * g.nwmax + p) * g.ntx;
            uint8_t *nrow = G.need_row.data() + ((size_t)b * g.nwmax + p) * g.ntx;
            for (int tu = 0; tu < g.ntx; ++tu)
                for (int tv = 0; tv < g.nty; ++tv) {
                    orow[tu] |= o[tu * g.nty + tv];
                    nrow[tu] |= nd[tu * g.nty + tv];
                }
        }
        std::stable_sort(gw.begin(), gw.end(), [](auto &a, auto &b) { return a.first > b.first; });
        std::stable_sort(iw.begin(), iw.end(), [](auto &a, auto &b) { return a.first > b.first; });
        for (auto &x : gw) G.gwork.push_back(x.second);
        for (auto &x : iw) G.iwork.push_back(x.second);
        G.gband_start[b + 1] = (int)G.gwork.size();
        G.iband_start[b + 1] = (int)G.iwork.size();
    }
    G.occ_list.clear();
    G.need_list.clear();
    G.occ_list_start.assign(g.n_band + 1, 0);
    G.need_list_start.assign(g.n_band + 1, 0);
    for (int b = 0; b < g.n_band; ++b) {
        for (int p = 0; p < g.nwmax; ++p)
            for (int tu = 0; tu < g.ntx; ++tu) {
                const size_t k = ((size_t)b * g.nwmax + p) * g.ntx + tu;
                if (G.occ_row[k]) G.occ_list.push_back((int32_t)k);
                if (G.need_row[k]) G.need_list.push_back((int32_t)k);
            }
        G.occ_list_start[b + 1] = (int)G.occ_list.size();
        G.need_list_start[b + 1] = (int)G.need_list.size();
    }
}

// Installs the plan's launch profiler for the duration of one operator call.
struct ProfScope {
    explicit ProfScope(pfb_plan *P) {
        if (P && P->prof_on) set_thread_profiler(&P->prof);
    }
    ~ProfScope() { set_thread_profiler(nullptr); }
};

pfb_status check_ready(const pfb_plan *P) {
    if (!P) return fail(PFB_EINVAL, "plan is NULL");
    if (!P->ws_ready) return fail(PFB_ESTATE, "pfb_plan_set_workspace has not been called");
    return PFB_OK;
}

XformArgs xform_args(const pfb_plan *P, const GridderHost &G, int b0, int nbb) {
    XformArgs a{};
    a.g = G.g;
    a.bands = G.d_bands;
    a.band0 = b0;
    a.n_bb = nbb;
    a.tw = P->p(P->o_tw);
    a.log2_lmax = P->log2_lmax;
    a.planes = P->p(P->o_planes);
    a.t1 = P->p(P->o_t1);
    a.corr2d = G.corr2d ? G.d_corr2d : nullptr;
    a.corr_x = G.d_corrx;
    a.corr_y = G.d_corry;
    a.occ = G.d_occ;
    a.need = G.d_need;
    a.occ_row = G.d_occ_row;
    a.need_row = G.d_need_row;
    a.occ_list = G.d_occ_list + G.occ_list_start[b0];
    a.n_occ_list = G.occ_list_start[b0 + nbb] - G.occ_list_start[b0];
    a.need_list = G.d_need_list + G.need_list_start[b0];
    a.n_need_list = G.need_list_start[b0 + nbb] - G.need_list_start[b0];
    return a;
}

ConvArgs conv_args(const pfb_plan *P) {
    ConvArgs a{};
    a.n_band = P->prob.n_band;
    a.nx = P->prob.nx;
    a.lx = P->conv_lx;
    a.ly = P->conv_ly;
    a.ny = P->prob.ny;
    a.ldh = P->ldh;
    a.cgc = P->conv_cgc;
    a.tw = P->p(P->o_tw);
    a.log2_lmax = P->log2_lmax;
    a.t1c = P->p(P->o_t1c);
    a.psfhat = P->p(P->o_psfhat);
    a.partials = reinterpret_cast<double *>(P->p(P->o_partials));
    a.max_partials = P->max_partials;
    a.scal = reinterpret_cast<double *>(P->p(P->o_scal));
    return a;
}

// FP32 path: max |z| of the values to be spread (scale of the fixed-point LDS accumulators)
pfb_status spread_prepass(pfb_plan *P, int vmode, const void *vis, hipStream_t s) {
    if (P->dbl) return PFB_OK;
    float *buf = reinterpret_cast<float *>(P->p(P->o_absmax));
    hipError_t e = launch_absmax(vmode, vis, P->prob.weight, P->prob.flag, P->prob.n_row * P->prob.n_chan,
                                 buf + 64, buf, s);
    if (e != hipSuccess) return fail(PFB_EHIP, "absmax pre-pass: %s", hipGetErrorString(e));
    return PFB_OK;
}

SpreadLaunch spread_args(const pfb_plan *P, const GridderHost &G, int b0, int nbb, int vmode, const void *vis,
                         void *planes) {
    SpreadLaunch s{};
    s.absmax = reinterpret_cast<const float *>(P->p(P->o_absmax));
    s.g = G.g;
    s.bands = G.d_bands;
    s.work = G.d_gwork + G.gband_start[b0];
    s.n_work = G.gband_start[b0 + nbb] - G.gband_start[b0];
    s.offsets = G.d_offsets;
    s.recs = G.d_recs;
    s.omega = G.d_omega;
    s.phase = G.mfma ? G.d_phase : nullptr;
    s.vis = vis;
    s.planes = planes;
    s.band0 = b0;
    s.vmode = vmode;
    s.home_pos = G.d_home_pos;
    return s;
}

InterpLaunch interp_args(const GridderHost &G, int b0, int nbb, int omode, const void *planes, void *out) {
    InterpLaunch s{};
    s.g = G.g;
    s.bands = G.d_bands;
    s.work = G.d_iwork + G.iband_start[b0];
    s.n_work = G.iband_start[b0 + nbb] - G.iband_start[b0];
    s.offsets = G.d_offsets;
    s.recs = G.d_recs;
    s.omega = G.d_omega;
    s.planes = planes;
    s.out = out;
    s.band0 = b0;
    s.omode = omode;
    s.phase = G.mfma ? G.d_phase : nullptr;
    s.use_phase = G.mfma && (G.g.offx || G.g.offy);
    s.hidx = G.d_hidx;
    s.hoffsets = G.d_hoffsets;
    return s;
}

#define LAUNCH_OK(expr)                                                                  \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return fail(PFB_EHIP, "%s: %s", #expr, hipGetErrorString(_e));              \
    } while (0)

// tol > 0: after every iteration the squared residuals are read back (host
// synchronisation) and the loop stops once every band has |r| <= tol |g|.
pfb_status cg_solve(pfb_plan *P, const void *g, void *y, double sigma, int iters, hipStream_t s, double tol = 0.0,
                    int *iters_done = nullptr) {
    const bool d = P->dbl;
    ConvArgs ca = conv_args(P);
    const int nb = P->prob.n_band;
    const int64_t Pn = (int64_t)P->prob.nx * P->prob.ny;
    char *v = reinterpret_cast<char *>(P->p(P->o_vec));
    void *r = v, *p = v + P->vec_bytes, *ap = v + 2 * P->vec_bytes;
    const int vparts = vec_partials_per_band(Pn);
    const int cparts = conv_partials_per_band(d, ca);
    LAUNCH_OK(launch_vec(d, VEC_CG_INIT, nb, Pn, ca.partials, ca.max_partials, ca.scal, const_cast<void *>(g), y, r,
                         p, nullptr, 0, 0, s));
    LAUNCH_OK(launch_reduce(RED_SET_RR, nb, ca.partials, vparts, ca.max_partials, ca.scal, s));
    for (int it = 0; it < iters; ++it) {
        LAUNCH_OK(launch_psf_conv(d, ca, r, p, ap, p, sigma, CONV_IN_CG_P, CONV_OUT_CG, s));
        LAUNCH_OK(launch_reduce(RED_ALPHA, nb, ca.partials, cparts, ca.max_partials, ca.scal, s));
        LAUNCH_OK(launch_vec(d, VEC_CG_UPDATE, nb, Pn, ca.partials, ca.max_partials, ca.scal, nullptr, y, r, p, ap,
                             0, 0, s));
        LAUNCH_OK(launch_reduce(RED_BETA, nb, ca.partials, vparts, ca.max_partials, ca.scal, s));
        if (iters_done) *iters_done = it + 1;
        if (tol > 0.0) {
            std::vector<double> sc((size_t)nb * 8);
            HIP_OK(hipMemcpyAsync(sc.data(), ca.scal, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            bool done = true;
            for (int b = 0; b < nb; ++b) done = done && sc[(size_t)b * 8 + S_RR] <= tol * tol * sc[(size_t)b * 8 + S_RR0];
            if (done) break;
        }
    }
    return PFB_OK;
}

pfb_status hessian_impl(pfb_plan *P, const void *x, void *y, hipStream_t s) {
    const bool d = P->dbl;
    GridderHost &G = P->main;
    for (int b0 = 0; b0 < P->prob.n_band; b0 += P->band_batch) {
        const int nbb = std::min(P->band_batch, P->prob.n_band - b0);
        XformArgs xa = xform_args(P, G, b0, nbb);
        xa.image_in = x;
        xa.image_out = y;
        LAUNCH_OK(launch_degrid_xform(d, xa, s));
        InterpLaunch ia = interp_args(G, b0, nbb, 1, P->p(P->o_planes), P->p(P->o_vals));
        if (!d) {   // FP32: the interpolation also finds the fixed-point scale of the spread
            ia.absmax = reinterpret_cast<float *>(P->p(P->o_absmax));
            LAUNCH_OK(launch_absmax_clear(ia.absmax, s));
        }
        LAUNCH_OK(launch_interp(d, ia, s));
        LAUNCH_OK(launch_spread(d, spread_args(P, G, b0, nbb, 2, P->p(P->o_vals), P->p(P->o_planes)), s));
        LAUNCH_OK(launch_grid_xform(d, xa, s));
    }
    return PFB_OK;
}


// Bytes of the counting scratch of pfb_plan_count: the channel tables, both
// gridders' band descriptors, ONE band's (tile, base plane) counters of both
// gridders (bands are counted one after another) and the global counters.
struct CountLayout {
    size_t freq, cb, bm, bq, cm, cq, hm, hq, ctr, total;
    int64_t kMb, kQb;   // keys per band of the main and the PSF gridder
};
CountLayout count_layout(const pfb_plan &P) {
    CountLayout c{};
    const pfb_problem &pr = P.prob;
    c.kMb = P.main.keys() / pr.n_band;
    c.kQb = P.psf.keys() / pr.n_band;
    Layout tl;
    c.freq = tl.take(pr.n_chan * sizeof(double));
    c.cb = tl.take(pr.n_chan * sizeof(int));
    c.bm = tl.take(P.main.bands.size() * sizeof(BandDev));
    c.bq = tl.take(P.psf.bands.size() * sizeof(BandDev));
    c.cm = tl.take(c.kMb * sizeof(unsigned));
    c.cq = tl.take(c.kQb * sizeof(unsigned));
    c.hm = tl.take(c.kMb * sizeof(unsigned));
    c.hq = tl.take(c.kQb * sizeof(unsigned));
    c.ctr = tl.take(8 * sizeof(unsigned long long));
    c.total = tl.off;
    return c;
}

// Counting pass (per band, in `tmp`), then bucket offsets, work lists, tables and
// the workspace layout.  Synchronises `stream` once, after the last band.
pfb_status count_and_layout(pfb_plan *P, char *tmp, hipStream_t stream) {
    const pfb_problem &pr = P->prob;
    const pfb_options &opt = P->opt;
    const bool dbl = P->dbl;
    GridderHost &M = P->main;
    GridderHost &Q = P->psf;
    const CountLayout cl = count_layout(*P);
    const int64_t kM = M.keys(), kQ = Q.keys();
    std::vector<unsigned> cM(kM), cQ(kQ), hM(kM), hQ(kQ);
    unsigned long long ctr[8] = {0};
    std::vector<int> cb(P->chan_band.begin(), P->chan_band.end());
    pfb_status st = PFB_OK;
    do {
        hipError_t e = hipSuccess;
#define TMP_OK(x)                                                                    \
    e = (x);                                                                         \
    if (e != hipSuccess) {                                                           \
        st = fail(PFB_EHIP, "%s: %s", #x, hipGetErrorString(e));                    \
        break;                                                                       \
    }
        TMP_OK(hipMemcpyAsync(tmp + cl.freq, P->freq.data(), pr.n_chan * sizeof(double), hipMemcpyHostToDevice, stream));
        TMP_OK(hipMemcpyAsync(tmp + cl.cb, cb.data(), pr.n_chan * sizeof(int), hipMemcpyHostToDevice, stream));
        TMP_OK(hipMemcpyAsync(tmp + cl.bm, M.bands.data(), M.bands.size() * sizeof(BandDev), hipMemcpyHostToDevice, stream));
        TMP_OK(hipMemcpyAsync(tmp + cl.bq, Q.bands.data(), Q.bands.size() * sizeof(BandDev), hipMemcpyHostToDevice, stream));
        TMP_OK(hipMemsetAsync(tmp + cl.ctr, 0, 8 * sizeof(unsigned long long), stream));
        unsigned long long *c = reinterpret_cast<unsigned long long *>(tmp + cl.ctr);
        for (int b = 0; b < pr.n_band; ++b) {
            TMP_OK(hipMemsetAsync(tmp + cl.cm, 0, cl.kMb * sizeof(unsigned), stream));
            TMP_OK(hipMemsetAsync(tmp + cl.cq, 0, cl.kQb * sizeof(unsigned), stream));
            TMP_OK(hipMemsetAsync(tmp + cl.hm, 0, cl.kMb * sizeof(unsigned), stream));
            TMP_OK(hipMemsetAsync(tmp + cl.hq, 0, cl.kQb * sizeof(unsigned), stream));
            BucketArgs ba{};
            ba.uvw = pr.uvw;
            ba.freq_dev = reinterpret_cast<const double *>(tmp + cl.freq);
            ba.chan_band_dev = reinterpret_cast<const int *>(tmp + cl.cb);
            ba.weight = pr.weight;
            ba.flag = pr.flag;
            ba.n_row = pr.n_row;
            ba.n_chan = pr.n_chan;
            ba.band_sel = b;
            ba.g = M.g;
            ba.bands = reinterpret_cast<const BandDev *>(tmp + cl.bm);
            ba.counts = reinterpret_cast<unsigned *>(tmp + cl.cm);
            ba.home_counts = reinterpret_cast<unsigned *>(tmp + cl.hm);
            ba.n_active = c;
            ba.n_flagged = c + 1;
            ba.n_bad = c + 2;
            ba.n_badw = c + 6;
            TMP_OK(launch_count(dbl, ba, stream));
            ba.n_badw = nullptr;
            ba.g = Q.g;
            ba.bands = reinterpret_cast<const BandDev *>(tmp + cl.bq);
            ba.counts = reinterpret_cast<unsigned *>(tmp + cl.cq);
            ba.home_counts = reinterpret_cast<unsigned *>(tmp + cl.hq);
            ba.n_active = c + 3;
            ba.n_flagged = c + 4;
            ba.n_bad = c + 5;
            TMP_OK(launch_count(dbl, ba, stream));
            // stream order: each band's copies finish before the next band clears the counters
            TMP_OK(hipMemcpyAsync(cM.data() + b * cl.kMb, tmp + cl.cm, cl.kMb * sizeof(unsigned), hipMemcpyDeviceToHost, stream));
            TMP_OK(hipMemcpyAsync(cQ.data() + b * cl.kQb, tmp + cl.cq, cl.kQb * sizeof(unsigned), hipMemcpyDeviceToHost, stream));
            TMP_OK(hipMemcpyAsync(hM.data() + b * cl.kMb, tmp + cl.hm, cl.kMb * sizeof(unsigned), hipMemcpyDeviceToHost, stream));
            TMP_OK(hipMemcpyAsync(hQ.data() + b * cl.kQb, tmp + cl.hq, cl.kQb * sizeof(unsigned), hipMemcpyDeviceToHost, stream));
        }
        if (st != PFB_OK) break;
        TMP_OK(hipMemcpyAsync(ctr, c, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
        TMP_OK(hipStreamSynchronize(stream));
#undef TMP_OK
    } while (0);
    if (st != PFB_OK) return st;
    if (ctr[6])
        return fail(PFB_EINVAL, "%llu unflagged weights are NaN, negative or infinite (weights are diag(Sigma^-1) >= 0)",
                    ctr[6]);
    if (ctr[2] || ctr[5]) return fail(PFB_EINVAL, "%llu visibilities fell outside the planned w range", ctr[2] + ctr[5]);
    P->n_active = (int64_t)ctr[0];
    P->n_flagged = (int64_t)ctr[1];
    // bucket offsets and work lists
    for (GridderHost *G : {&M, &Q}) {
        const std::vector<unsigned> &cnt = (G == &M) ? cM : cQ;
        G->offsets.resize(cnt.size() + 1);
        int64_t acc = 0;
        for (size_t k = 0; k < cnt.size(); ++k) {
            G->offsets[k] = acc;
            acc += cnt[k];
        }
        G->offsets[cnt.size()] = acc;
        G->n_entries = acc;
        const std::vector<unsigned> &hcnt = (G == &M) ? hM : hQ;
        G->hoffsets.resize(hcnt.size() + 1);
        int64_t hacc = 0;
        for (size_t k = 0; k < hcnt.size(); ++k) {
            G->hoffsets[k] = hacc;
            hacc += hcnt[k];
        }
        G->hoffsets[hcnt.size()] = hacc;
        G->n_home = hacc;
        if (acc >= (int64_t(1) << 31)) {
            fail(PFB_EUNSUPPORTED, "%lld bucket entries exceed 2^31", (long long)acc);
            return PFB_EUNSUPPORTED;
        }
        // work-item size: a given chunk, else one compute unit's share of all entries
        // (>= 4096): a spread item split by plane range re-reads the entries of the
        // W - 1 base planes its neighbour also covers, so only tiles heavier than a
        // unit's share are split
        int n_cu = 0;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
            n_cu = 256;
        const int chunk = opt.chunk ? opt.chunk
                                    : (int)std::min<int64_t>(std::max<int64_t>(4096, acc / n_cu), 1 << 24);
        build_work(*G, cnt, hcnt, chunk);
        G->sort_items.clear();
        for (size_t k2 = 0; k2 < cnt.size(); ++k2)
            if (cnt[k2]) {
                G->sort_items.push_back(G->offsets[k2]);
                G->sort_items.push_back(cnt[k2]);
                G->sort_items.push_back((int64_t)(k2 / ((size_t)G->g.ntx * G->g.nty * G->g.nj0max)));
                G->sort_items.push_back((int64_t)k2);
            }
        if (sort_key_bits(G->keys(), G->g.T, G->g.W, G->sort_rb, G->sort_cb, pr.n_row * pr.n_chan) > 64) {
            fail(PFB_EUNSUPPORTED, "bucket sort key exceeds 64 bits (too many buckets x visibilities)");
            return PFB_EUNSUPPORTED;
        }
    }

    // grid correction: Chebyshev expansion of the ES kernel's Fourier transform
    {
        PsiHat ph(opt.support, M.g.beta);
        double err = 0.0;
        P->cheb = psihat_chebyshev(ph, P->xi_max, 40, &err);
        if (err > 1e-13) {
            fail(PFB_EHIP, "correction expansion error %.3g too large", err);
            return PFB_EHIP;
        }
    }
    // twiddles
    const int lmax = std::max({Q.g.gx, Q.g.gy, M.g.gx, M.g.gy});
    P->log2_lmax = ilog2(lmax);
    P->tw_host.resize(2 * (size_t)lmax);
    for (int e2 = 0; e2 < lmax; ++e2) {
        const double a = -2.0 * M_PI * (double)e2 / lmax;
        P->tw_host[2 * e2] = std::cos(a);
        P->tw_host[2 * e2 + 1] = std::sin(a);
    }
    // zero-padded grid of the PSF convolution: powers of two >= 2 nx, 2 ny
    P->conv_lx = next_pow2(2 * (int64_t)pr.nx);
    P->conv_ly = next_pow2(2 * (int64_t)pr.ny);
    P->conv_cgc = conv_group_cols(dbl, P->conv_lx / 2);
    P->ldh = ((P->conv_ly / 2 + 1 + 15) / 16) * 16;

    // band batch
    P->band_batch = opt.band_batch > 0 ? std::min(opt.band_batch, pr.n_band) : pr.n_band;
    const size_t csz = 2 * P->rsz;
    const size_t per_band_planes = std::max((size_t)M.g.nwmax * M.g.gx * M.g.gy, (size_t)Q.g.gx * Q.g.gy) * csz;
    if (opt.band_batch == 0) {
        const size_t budget = (size_t)160 << 30;  // planes + two intermediates (MI355X: 288 GB HBM)
        while (P->band_batch > 1 && P->band_batch * 2 * per_band_planes > budget) --P->band_batch;
    }
    P->opt.band_batch = P->band_batch;

    // workspace layout
    Layout L;
    const int nb = pr.n_band;
    const size_t Pimg = (size_t)pr.nx * pr.ny;
    P->o_freq = L.take(pr.n_chan * sizeof(double));
    P->o_cb = L.take(pr.n_chan * sizeof(int));
    P->o_cheb = L.take(P->cheb.size() * sizeof(double));
    P->o_tw = L.take((size_t)lmax * csz);
    P->o_flagged = L.take(std::max<int64_t>(P->n_flagged, 1) * sizeof(uint32_t));
    P->o_flagcur = L.take(sizeof(unsigned long long));
    for (GridderHost *G : {&M, &Q}) {
        G->o_bands = L.take(G->bands.size() * sizeof(BandDev));
        G->o_offsets = L.take(G->offsets.size() * sizeof(int64_t));
        G->o_cursor = L.take((G->offsets.size()) * sizeof(unsigned long long));
        G->o_gwork = L.take(std::max<size_t>(G->gwork.size(), 1) * sizeof(GridWork));
        G->o_iwork = L.take(std::max<size_t>(G->iwork.size(), 1) * sizeof(InterpWork));
        G->o_sortitems = L.take(std::max<size_t>(G->sort_items.size(), 4) * sizeof(int64_t));
        G->o_recs = L.take(std::max<int64_t>(G->n_entries, 1) * (dbl ? sizeof(Rec<double>) : sizeof(Rec<float>)));
        G->o_omega = L.take(std::max<int64_t>(G->n_entries, 1) * P->rsz);
        G->o_hoffsets = L.take(G->hoffsets.size() * sizeof(int64_t));
        G->o_hidx = L.take(std::max<int64_t>(G->n_home, 1) * sizeof(uint32_t));
        if (G->mfma) G->o_phase = L.take(std::max<int64_t>(G->n_entries, 1) * 2 * sizeof(float));
        if (G == &M) G->o_home_pos = L.take(std::max<int64_t>(G->n_entries, 1) * sizeof(uint32_t));
        G->o_occ = L.take(std::max<size_t>(G->occ.size(), 1));
        G->o_need = L.take(std::max<size_t>(G->need.size(), 1));
        G->o_occ_row = L.take(std::max<size_t>(G->occ_row.size(), 1));
        G->o_need_row = L.take(std::max<size_t>(G->need_row.size(), 1));
        G->o_occ_list = L.take(std::max<size_t>(G->occ_list.size(), 1) * sizeof(int32_t));
        G->o_need_list = L.take(std::max<size_t>(G->need_list.size(), 1) * sizeof(int32_t));
        if (G->corr2d) {
            G->o_corr2d = L.take((size_t)nb * G->g.nx * G->g.ny * P->rsz);
        } else {
            G->o_corrx = L.take((size_t)G->g.nx * P->rsz);
            G->o_corry = L.take((size_t)G->g.ny * P->rsz);
        }
    }
    P->planes_bytes = (size_t)P->band_batch * per_band_planes;
    {
        // cropped row spectra, columns padded to whole groups of plane_group_cols
        const size_t cg = (size_t)plane_group_cols(dbl);
        auto padded = [cg](int n) { return ((size_t)n + cg - 1) / cg * cg; };
        P->t_bytes = (size_t)P->band_batch *
                     std::max((size_t)M.g.nwmax * M.g.gx * padded(M.g.ny), (size_t)Q.g.gx * padded(Q.g.ny)) * csz;
    }
    P->o_planes = L.take(P->planes_bytes);
    P->o_t1 = L.take(P->t_bytes);
    {
        const size_t recsz = dbl ? sizeof(Rec<double>) : sizeof(Rec<float>);
        size_t need = 0;
        for (GridderHost *G : {&M, &Q})
            need = std::max(need, (((size_t)G->n_entries * recsz + 255) & ~size_t(255)) +
                                      (((size_t)G->n_entries * P->rsz + 255) & ~size_t(255)) +
                                      sort_scratch_bytes(G->n_entries));
        P->o_sorttmp = (L.off - P->o_planes >= need) ? P->o_planes : L.take(need);
    }
    P->o_vals = L.take((size_t)pr.n_row * pr.n_chan * csz);
    P->o_psfimg = L.take((size_t)nb * 4 * Pimg * P->rsz);
    P->o_t1c = L.take((size_t)nb * P->conv_lx * P->ldh * csz);
    P->o_psfhat = L.take((size_t)nb * P->conv_lx * P->ldh * P->rsz);
    P->vec_bytes = ((Pimg * nb * P->rsz) + 255) & ~size_t(255);
    P->o_vec = L.take(6 * P->vec_bytes);
    {
        ConvArgs ca{};
        ca.nx = pr.nx;
        ca.ny = pr.ny;
        ca.lx = P->conv_lx;
        ca.ly = P->conv_ly;
        P->max_partials = std::max(vec_partials_per_band((int64_t)Pimg), conv_partials_per_band(dbl, ca));
    }
    P->o_partials = L.take((size_t)nb * P->max_partials * sizeof(double));
    P->o_scal = L.take((size_t)nb * 8 * sizeof(double));
    P->o_absmax = L.take((kAbsmaxBlocks + 64) * sizeof(float));
    P->ws_bytes = L.off;
    P->counted = true;
    return PFB_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *pfb_last_error(void) { return g_last_error.c_str(); }
const char *pfb_version(void) { return "pfb-mi355x 0.1 (gfx950)"; }

pfb_status pfb_plan_create(pfb_plan **out, const pfb_problem *prob, const pfb_options *opt_in, hipStream_t stream) {
    if (!out) return fail(PFB_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    if (!prob) return fail(PFB_EINVAL, "problem is NULL");
    pfb_options opt{};
    if (opt_in) opt = *opt_in;
    const pfb_problem &pr = *prob;
    if (pr.n_row <= 0 || pr.n_chan <= 0 || pr.n_band <= 0)
        return fail(PFB_EINVAL, "n_row, n_chan and n_band must be positive");
    if (pr.n_band > pr.n_chan) return fail(PFB_EINVAL, "more bands than channels");
    if (pr.n_row * pr.n_chan >= (int64_t(1) << 31))
        return fail(PFB_EUNSUPPORTED, "n_row * n_chan must be below 2^31");
    if (!pr.chan_band || !pr.freq || !pr.uvw || !pr.weight) return fail(PFB_EINVAL, "NULL array in problem");
    if ((pr.nx & 1) || (pr.ny & 1) || pr.nx < 16 || pr.ny < 16)
        return fail(PFB_EINVAL, "nx and ny must be even and >= 16 (got %d x %d)", pr.nx, pr.ny);
    if (!(pr.cellx > 0) || !(pr.celly > 0) || !std::isfinite(pr.cellx) || !std::isfinite(pr.celly))
        return fail(PFB_EINVAL, "cell sizes must be positive and finite");
    if (opt.precision != PFB_FP32 && opt.precision != PFB_FP64) return fail(PFB_EINVAL, "unknown precision");
    const bool dbl = opt.precision == PFB_FP64;
    if (!(opt.epsilon >= 0.0) || !std::isfinite(opt.epsilon)) return fail(PFB_EINVAL, "epsilon must be finite and >= 0");
    if (opt.support == 0 && opt.epsilon > 0.0) {
        // rel-l2 error of the 1-D ES NUFFT at sigma = 2, beta = 2.30 W (W = 6..8 and
        // 11..13 measured, the rest geometric inter- and extrapolation); the 3-D product
        // kernel (u, v, w) is taken as three times that, plus the rounding floor of the
        // arithmetic (FP32 path: 2e-6, the largest error measured at W = 8; FP64: 1e-14)
        static const double err1d[17] = {0, 0, 0, 0, 6.0e-4, 6.8e-5, 7.7e-6, 8.8e-7, 1.0e-7,
                                         1.2e-8, 1.4e-9, 1.8e-10, 1.7e-11, 1.7e-12, 1.7e-13, 1.7e-14, 1.7e-15};
        const int wlo = dbl ? 9 : 4, whi = dbl ? 16 : 8;
        const double floor_err = dbl ? 1e-14 : 2e-6;
        for (int W = wlo; W <= whi && opt.support == 0; ++W)
            if (3.0 * err1d[W] + floor_err <= opt.epsilon) opt.support = W;
        if (opt.support == 0)
            return fail(PFB_EINVAL, "epsilon %.3g is below what the %s path reaches (%.1e)", opt.epsilon,
                        dbl ? "FP64" : "FP32", 3.0 * err1d[whi] + floor_err);
    }
    if (opt.support == 0) opt.support = dbl ? 13 : 7;
    if (dbl ? (opt.support < 9 || opt.support > 16) : (opt.support < 4 || opt.support > 8))
        return fail(PFB_EINVAL, "support %d outside the range compiled for this precision", opt.support);
    if (opt.oversample == 0.0) opt.oversample = 2.0;
    if (opt.oversample != 2.0) return fail(PFB_EUNSUPPORTED, "only oversampling 2.0 is implemented");
    if (opt.tile == 0) opt.tile = std::max(8, std::min(dbl ? 8 : 32, std::min(pr.nx, pr.ny)));
    if (!is_pow2(opt.tile) || opt.tile < 8 || opt.tile > 64)
        return fail(PFB_EINVAL, "tile must be a power of two in [8, 64]");
    if (std::min(next_pow2(2 * (int64_t)pr.nx), next_pow2(2 * (int64_t)pr.ny)) < 2 * opt.tile)
        return fail(PFB_EINVAL, "tile larger than half the grid");
    if (gridder_lds_bytes(dbl, opt.support, opt.tile, opt.flat != 0) > kMaxLdsBytes)
        return fail(PFB_EINVAL, "tile %d with support %d needs %zu bytes of LDS per block (at most %zu)", opt.tile,
                    opt.support, gridder_lds_bytes(dbl, opt.support, opt.tile, opt.flat != 0), kMaxLdsBytes);
    if (opt.flat != 0 && opt.flat != 1) return fail(PFB_EINVAL, "flat must be 0 or 1");
    if (opt.chunk != 0 && opt.chunk < 64) return fail(PFB_EINVAL, "chunk must be >= 64");
    // FFT length limits (LDS-resident rows): the operator's grid rows have 2n points,
    // the PSF gridder's (a 2n x 2n image) 4n; in FP64 the latter stop at n = 2048, so
    // larger FP64 plans serve grid, degrid and the Hessian but not the PSF
    const int max_row = dbl ? 8192 : 16384;
    if (next_pow2(2 * (int64_t)pr.nx) > max_row || next_pow2(2 * (int64_t)pr.ny) > max_row)
        return fail(PFB_EUNSUPPORTED, "image %d x %d needs FFT rows longer than %d for this precision", pr.nx, pr.ny,
                    max_row);
    if ((pr.offx || pr.offy) && (dbl || opt.flat))
        return fail(PFB_EUNSUPPORTED, "facet offsets need the FP32 w-stacked path (not FP64, not flat)");
    if (std::abs((int64_t)pr.offx) > (int64_t)1 << 24 || std::abs((int64_t)pr.offy) > (int64_t)1 << 24)
        return fail(PFB_EINVAL, "facet offset out of range");
    // extreme l^2 + m^2 over the pixels: pixel i sits at l = (i - nx/2 + offx) cellx
    auto axis_range = [](int n, int off, double cell, double *amin, double *amax) {
        const double lo = (double)(off - n / 2) * cell, hi = (double)(off + n / 2 - 1) * cell;
        *amax = std::max(std::fabs(lo), std::fabs(hi));
        *amin = (lo <= 0.0 && hi >= 0.0) ? 0.0 : std::min(std::fabs(lo), std::fabs(hi));
    };
    double lmin_abs, lmax_abs, mmin_abs, mmax_abs;
    axis_range(pr.nx, pr.offx, pr.cellx, &lmin_abs, &lmax_abs);
    axis_range(pr.ny, pr.offy, pr.celly, &mmin_abs, &mmax_abs);
    const double lmax2 = lmax_abs * lmax_abs + mmax_abs * mmax_abs;
    const double lmin2 = lmin_abs * lmin_abs + mmin_abs * mmin_abs;
    if (!opt.flat && lmax2 >= 1.0) return fail(PFB_EINVAL, "field of view reaches l^2 + m^2 >= 1");

    pfb_plan *P = new pfb_plan();
    P->prob = pr;
    P->opt = opt;
    P->dbl = dbl;
    P->rsz = dbl ? 8 : 4;
    P->chan_band.assign(pr.chan_band, pr.chan_band + pr.n_chan);
    P->freq.assign(pr.freq, pr.freq + pr.n_chan);
    auto bail = [&](pfb_status st) {
        delete P;
        return st;
    };
    for (int64_t c = 0; c < pr.n_chan; ++c) {
        if (P->chan_band[c] < 0 || P->chan_band[c] >= pr.n_band) {
            fail(PFB_EINVAL, "chan_band[%lld] = %d outside [0, %d)", (long long)c, P->chan_band[c], pr.n_band);
            return bail(PFB_EINVAL);
        }
        if (!(P->freq[c] > 0) || !std::isfinite(P->freq[c])) {
            fail(PFB_EINVAL, "freq[%lld] is not a positive finite number", (long long)c);
            return bail(PFB_EINVAL);
        }
    }
    // uvw analysis on the host
    std::vector<double> uvw(3 * pr.n_row);
    {
        hipError_t e = hipMemcpyAsync(uvw.data(), pr.uvw, uvw.size() * sizeof(double), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            fail(PFB_EHIP, "copying uvw to the host failed: %s", hipGetErrorString(e));
            return bail(PFB_EHIP);
        }
    }
    double wlo = INFINITY, whi = -INFINITY;
    for (int64_t r = 0; r < pr.n_row; ++r) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(uvw[3 * r + k])) {
                fail(PFB_EINVAL, "uvw[%lld] is not finite", (long long)r);
                return bail(PFB_EINVAL);
            }
        wlo = std::min(wlo, uvw[3 * r + 2]);
        whi = std::max(whi, uvw[3 * r + 2]);
    }
    std::vector<double> fmin(pr.n_band, INFINITY), fmax(pr.n_band, 0.0);
    for (int64_t c = 0; c < pr.n_chan; ++c) {
        fmin[P->chan_band[c]] = std::min(fmin[P->chan_band[c]], P->freq[c]);
        fmax[P->chan_band[c]] = std::max(fmax[P->chan_band[c]], P->freq[c]);
    }

    // geometry of the two gridders
    GridderHost &M = P->main;
    M.g = base_geom(*P, pr.nx, pr.ny, opt.flat != 0);
    // n - 1 over the pixels lies in [s_min, s_max] (s_max = 0 when the image holds the
    // phase centre; a facet away from it has a narrower range and so fewer w-planes)
    P->s_min = opt.flat ? 0.0 : -lmax2 / (1.0 + std::sqrt(1.0 - lmax2));
    P->s_max = opt.flat ? 0.0 : -lmin2 / (1.0 + std::sqrt(1.0 - lmin2));
    M.bands.resize(pr.n_band);
    M.g.nj0max = 1;
    M.g.nwmax = 1;
    for (int b = 0; b < pr.n_band; ++b) {
        BandDev &bd = M.bands[b];
        if (opt.flat || P->s_max - P->s_min <= 0.0 || fmax[b] == 0.0) {
            bd.w0 = 0.0;
            bd.dw = 1.0;
            bd.sc = 0.0;
            bd.nw = 1;
            bd.nj0 = 1;
        } else {
            const double s0 = fmin[b] / kC0, s1 = fmax[b] / kC0;
            const double wmin = std::min({wlo * s0, wlo * s1, whi * s0, whi * s1});
            const double wmax = std::max({wlo * s0, wlo * s1, whi * s0, whi * s1});
            // w oversampling 2: |dw (s - sc)| <= 1/4 over the pixels
            bd.dw = 1.0 / (2.0 * (P->s_max - P->s_min));
            bd.sc = 0.5 * (P->s_min + P->s_max);
            const double D = (wmax - wmin) / bd.dw;
            bd.nj0 = (int)std::floor(D) + 2;
            bd.nw = bd.nj0 + opt.support - 1;
            bd.w0 = wmin - (0.5 * opt.support - 0.5) * bd.dw;
        }
        M.g.nj0max = std::max(M.g.nj0max, bd.nj0);
        M.g.nwmax = std::max(M.g.nwmax, bd.nw);
    }
    M.mfma = !dbl && !opt.flat;
    if (M.mfma) mfma_window(opt.support, &M.sort_rb, &M.sort_cb);
    GridderHost &Q = P->psf;
    Q.g = base_geom(*P, 2 * pr.nx, 2 * pr.ny, true);
    Q.bands.assign(pr.n_band, BandDev{0.0, 1.0, 0.0, 1, 1});
    Q.g.nj0max = 1;
    Q.g.nwmax = 1;
    Q.corr2d = false;

    *out = P;
    return PFB_OK;
}

pfb_status pfb_plan_count_scratch_size(const pfb_plan *P, size_t *bytes) {
    if (!P || !bytes) return fail(PFB_EINVAL, "NULL argument");
    *bytes = count_layout(*P).total;
    return PFB_OK;
}

pfb_status pfb_plan_count(pfb_plan *P, void *scratch, size_t bytes, hipStream_t stream) {
    if (!P) return fail(PFB_EINVAL, "plan is NULL");
    if (P->counted) return fail(PFB_ESTATE, "the plan has already been counted");
    const CountLayout cl = count_layout(*P);
    if (!scratch) return fail(PFB_EINVAL, "count scratch is NULL");
    if (bytes < cl.total) return fail(PFB_ENOMEM, "count scratch of %zu bytes < required %zu", bytes, cl.total);
    if (reinterpret_cast<uintptr_t>(scratch) & 255) return fail(PFB_EINVAL, "count scratch must be 256-byte aligned");
    return count_and_layout(P, reinterpret_cast<char *>(scratch), stream);
}

pfb_status pfb_plan_count_static(pfb_plan *P, hipStream_t stream) {
    if (!P) return fail(PFB_EINVAL, "plan is NULL");
    if (P->counted) return fail(PFB_ESTATE, "the plan has already been counted");
    const CountLayout cl = count_layout(*P);
    if (cl.total > kStaticScratchBytes)
        return fail(PFB_ENOMEM, "the counting pass needs %zu bytes, more than the %zu of the library's fixed buffer "
                    "(use pfb_plan_count with a caller buffer)", cl.total, kStaticScratchBytes);
    void *buf = nullptr;
    hipError_t e = static_scratch(&buf);
    if (e != hipSuccess) return fail(PFB_EHIP, "looking up the fixed count buffer: %s", hipGetErrorString(e));
    return count_and_layout(P, reinterpret_cast<char *>(buf), stream);
}

pfb_status pfb_plan_workspace_size(const pfb_plan *P, size_t *bytes) {
    if (!P || !bytes) return fail(PFB_EINVAL, "NULL argument");
    if (!P->counted) return fail(PFB_ESTATE, "pfb_plan_count has not been called");
    *bytes = P->ws_bytes;
    return PFB_OK;
}

pfb_status pfb_plan_get_info(const pfb_plan *P, pfb_plan_info *info) {
    if (!P || !info) return fail(PFB_EINVAL, "NULL argument");
    if (!P->counted) return fail(PFB_ESTATE, "pfb_plan_count has not been called");
    std::memset(info, 0, sizeof(*info));
    info->grid_x = P->main.g.gx;
    info->grid_y = P->main.g.gy;
    info->psf_grid_x = P->psf.g.gx;
    info->psf_grid_y = P->psf.g.gy;
    info->support = P->opt.support;
    info->tile = P->opt.tile;
    info->n_wplanes_max = P->main.g.nwmax;
    info->band_batch = P->band_batch;
    info->n_vis_active = P->n_active;
    info->n_entries = P->main.n_entries;
    info->n_psf_entries = P->psf.n_entries;
    info->s_min = P->s_min;
    info->s_max = P->s_max;
    info->es_beta = P->main.g.beta;
    info->workspace_bytes = (int64_t)P->ws_bytes;
    const GridderHost &G = P->main;
    const int ntiles = G.g.ntx * G.g.nty;
    for (int b = 0; b < G.g.n_band; ++b) {
        const int nw = G.g.flat ? 1 : G.bands[b].nw;
        info->n_wplanes_total += nw;
        for (int p = 0; p < nw; ++p) {
            const size_t base = ((size_t)b * G.g.nwmax + p) * ntiles;
            for (int tu = 0; tu < G.g.ntx; ++tu) {
                int no = 0, nn = 0;
                for (int tv = 0; tv < G.g.nty; ++tv) {
                    no += G.occ[base + (size_t)tu * G.g.nty + tv];
                    nn += G.need[base + (size_t)tu * G.g.nty + tv];
                }
                info->occ_tiles += no;
                info->need_tiles += nn;
                info->occ_tile_rows += no > 0;
                info->need_tile_rows += nn > 0;
            }
        }
    }
    return PFB_OK;
}

pfb_status pfb_plan_set_workspace(pfb_plan *P, void *dev, size_t bytes, hipStream_t s) {
    if (!P) return fail(PFB_EINVAL, "plan is NULL");
    if (!P->counted) return fail(PFB_ESTATE, "pfb_plan_count has not been called");
    if (!dev) return fail(PFB_ENOMEM, "workspace pointer is NULL");
    if (bytes < P->ws_bytes) return fail(PFB_ENOMEM, "workspace of %zu bytes < required %zu", bytes, P->ws_bytes);
    if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(PFB_EINVAL, "workspace must be 256-byte aligned");
    P->ws = reinterpret_cast<char *>(dev);
    P->ws_ready = false;
    P->psf_ready = false;
    const bool d = P->dbl;
    const pfb_problem &pr = P->prob;
    P->cb_host.assign(P->chan_band.begin(), P->chan_band.end());
    HIP_OK(hipMemcpyAsync(P->p(P->o_freq), P->freq.data(), pr.n_chan * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(P->p(P->o_cb), P->cb_host.data(), pr.n_chan * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(P->p(P->o_cheb), P->cheb.data(), P->cheb.size() * sizeof(double), hipMemcpyHostToDevice, s));
    {
        const size_t n = P->tw_host.size() / 2;
        if (d) {
            HIP_OK(hipMemcpyAsync(P->p(P->o_tw), P->tw_host.data(), n * 16, hipMemcpyHostToDevice, s));
        } else {
            P->tw_f32.assign(P->tw_host.begin(), P->tw_host.end());
            HIP_OK(hipMemcpyAsync(P->p(P->o_tw), P->tw_f32.data(), n * 8, hipMemcpyHostToDevice, s));
        }
    }
    HIP_OK(hipMemsetAsync(P->p(P->o_flagcur), 0, sizeof(unsigned long long), s));
    for (GridderHost *G : {&P->main, &P->psf}) {
        G->d_bands = reinterpret_cast<BandDev *>(P->p(G->o_bands));
        G->d_offsets = reinterpret_cast<int64_t *>(P->p(G->o_offsets));
        G->d_cursor = reinterpret_cast<unsigned long long *>(P->p(G->o_cursor));
        G->d_gwork = reinterpret_cast<GridWork *>(P->p(G->o_gwork));
        G->d_iwork = reinterpret_cast<InterpWork *>(P->p(G->o_iwork));
        G->d_recs = P->p(G->o_recs);
        G->d_omega = P->p(G->o_omega);
        G->d_phase = G->mfma ? P->p(G->o_phase) : nullptr;
        G->d_hidx = reinterpret_cast<uint32_t *>(P->p(G->o_hidx));
        G->d_hoffsets = reinterpret_cast<int64_t *>(P->p(G->o_hoffsets));
        G->d_occ = reinterpret_cast<const uint8_t *>(P->p(G->o_occ));
        G->d_need = reinterpret_cast<const uint8_t *>(P->p(G->o_need));
        HIP_OK(hipMemcpyAsync(P->p(G->o_occ), G->occ.data(), G->occ.size(), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(P->p(G->o_need), G->need.data(), G->need.size(), hipMemcpyHostToDevice, s));
        G->d_occ_row = reinterpret_cast<const uint8_t *>(P->p(G->o_occ_row));
        G->d_need_row = reinterpret_cast<const uint8_t *>(P->p(G->o_need_row));
        HIP_OK(hipMemcpyAsync(P->p(G->o_occ_row), G->occ_row.data(), G->occ_row.size(), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(P->p(G->o_need_row), G->need_row.data(), G->need_row.size(), hipMemcpyHostToDevice,
                              s));
        G->d_occ_list = reinterpret_cast<const int32_t *>(P->p(G->o_occ_list));
        G->d_need_list = reinterpret_cast<const int32_t *>(P->p(G->o_need_list));
        if (!G->occ_list.empty())
            HIP_OK(hipMemcpyAsync(P->p(G->o_occ_list), G->occ_list.data(), G->occ_list.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
        if (!G->need_list.empty())
            HIP_OK(hipMemcpyAsync(P->p(G->o_need_list), G->need_list.data(), G->need_list.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
        if (G->corr2d) {
            G->d_corr2d = P->p(G->o_corr2d);
        } else {
            G->d_corrx = P->p(G->o_corrx);
            G->d_corry = P->p(G->o_corry);
        }
        HIP_OK(hipMemcpyAsync(G->d_bands, G->bands.data(), G->bands.size() * sizeof(BandDev), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(G->d_hoffsets, G->hoffsets.data(), G->hoffsets.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(G->d_offsets, G->offsets.data(), G->offsets.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(G->d_cursor, G->d_offsets, G->offsets.size() * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, s));
        if (!G->gwork.empty())
            HIP_OK(hipMemcpyAsync(G->d_gwork, G->gwork.data(), G->gwork.size() * sizeof(GridWork),
                                  hipMemcpyHostToDevice, s));
        if (!G->iwork.empty())
            HIP_OK(hipMemcpyAsync(G->d_iwork, G->iwork.data(), G->iwork.size() * sizeof(InterpWork),
                                  hipMemcpyHostToDevice, s));
        if (!G->sort_items.empty())
            HIP_OK(hipMemcpyAsync(P->p(G->o_sortitems), G->sort_items.data(), G->sort_items.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, s));
        const size_t recsz = d ? sizeof(Rec<double>) : sizeof(Rec<float>);
        void *tmp_recs = P->p(P->o_sorttmp);
        const size_t tmp_rec_bytes = ((size_t)G->n_entries * recsz + 255) & ~size_t(255);
        void *tmp_om = P->p(P->o_sorttmp + tmp_rec_bytes);
        void *sort_scratch = P->p(P->o_sorttmp + tmp_rec_bytes + (((size_t)G->n_entries * P->rsz + 255) & ~size_t(255)));
        BucketArgs ba{};
        ba.g = G->g;
        ba.uvw = pr.uvw;
        ba.freq_dev = reinterpret_cast<const double *>(P->p(P->o_freq));
        ba.chan_band_dev = reinterpret_cast<const int *>(P->p(P->o_cb));
        ba.weight = pr.weight;
        ba.flag = pr.flag;
        ba.bands = G->d_bands;
        ba.n_row = pr.n_row;
        ba.n_chan = pr.n_chan;
        ba.cursor = G->d_cursor;
        ba.recs = tmp_recs;
        ba.omega = tmp_om;
        if (G == &P->main) {
            ba.flagged = reinterpret_cast<uint32_t *>(P->p(P->o_flagged));
            ba.flag_cursor = reinterpret_cast<unsigned long long *>(P->p(P->o_flagcur));
        }
        LAUNCH_OK(launch_scatter(d, ba, s));
        LAUNCH_OK(launch_sort(d, tmp_recs, tmp_om, G->d_recs, G->d_omega,
                              reinterpret_cast<const int64_t *>(P->p(G->o_sortitems)), (int)(G->sort_items.size() / 4),
                              G->n_entries, G->keys(), (int64_t)G->g.ntx * G->g.nty * G->g.nj0max,
                              pr.n_row * pr.n_chan, G->g.T, G->g.W, G->sort_rb, G->sort_cb, G->d_bands, G->g,
                              G->d_phase, sort_scratch, s));
        LAUNCH_OK(launch_home_list(d, G->d_recs, reinterpret_cast<const int64_t *>(P->p(G->o_sortitems)),
                                   (int)(G->sort_items.size() / 4), G->d_hoffsets, G->d_hidx, s));
        if (G == &P->main) {   // Hessian values travel in home-list order; o_vals is scratch here
            G->d_home_pos = reinterpret_cast<uint32_t *>(P->p(G->o_home_pos));
            LAUNCH_OK(launch_home_pos(d, G->d_recs, G->d_hidx, G->n_home, G->n_entries,
                                      reinterpret_cast<uint32_t *>(P->p(P->o_vals)), G->d_home_pos, s));
        }
        const double *cheb = reinterpret_cast<const double *>(P->p(P->o_cheb));
        const int nch = (int)P->cheb.size();
        if (G->corr2d) {
            LAUNCH_OK(launch_corr2d(d, G->g, G->d_bands, cheb, nch, P->xi_max, G->d_corr2d, s));
        } else {
            LAUNCH_OK(launch_corr1d(d, G->g.nx, G->g.gx, cheb, nch, P->xi_max, G->d_corrx, s));
            LAUNCH_OK(launch_corr1d(d, G->g.ny, G->g.gy, cheb, nch, P->xi_max, G->d_corry, s));
        }
    }
    HIP_OK(hipMemsetAsync(P->p(P->o_scal), 0, (size_t)pr.n_band * 8 * sizeof(double), s));
    // per-visibility Hessian values: keep entries that no band batch writes finite
    HIP_OK(hipMemsetAsync(P->p(P->o_vals), 0, (size_t)pr.n_row * pr.n_chan * 2 * P->rsz, s));
    P->ws_ready = true;
    return PFB_OK;
}

pfb_status pfb_plan_destroy(pfb_plan *P) {
    delete P;
    return PFB_OK;
}

}  // extern "C"

struct pfb_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~pfb_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

extern "C" {

pfb_status pfb_fb_graph_create(pfb_plan *P, const void *dirty, void *x, double sigma, double gamma, double lambda,
                               int cg_iters, int n_steps, hipStream_t s, pfb_graph **out) {
    if (!out) return fail(PFB_EINVAL, "graph output pointer is NULL");
    *out = nullptr;
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!s) return fail(PFB_EINVAL, "capture needs a non-default stream");
    if (n_steps < 1) return fail(PFB_EINVAL, "n_steps must be >= 1");
    if (P->prof_on) return fail(PFB_ESTATE, "disable profiling before capturing a graph");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < n_steps && st == PFB_OK; ++k) st = pfb_fb_step(P, dirty, x, sigma, gamma, lambda, cg_iters, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != PFB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(PFB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    pfb_graph *G = new pfb_graph();
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        delete G;
        return fail(PFB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = G;
    return PFB_OK;
}

pfb_status pfb_graph_launch(pfb_graph *G, hipStream_t s) {
    if (!G || !G->exec) return fail(PFB_EINVAL, "graph is NULL");
    HIP_OK(hipGraphLaunch(G->exec, s));
    return PFB_OK;
}

pfb_status pfb_graph_destroy(pfb_graph *G) {
    delete G;
    return PFB_OK;
}

pfb_status pfb_profile_enable(pfb_plan *P, int on) {
    if (!P) return fail(PFB_EINVAL, "plan is NULL");
    if (on) P->prof.clear();
    P->prof_on = on != 0;
    return PFB_OK;
}

pfb_status pfb_profile_report(pfb_plan *P, char *buf, size_t len) {
    if (!P || !buf || len == 0) return fail(PFB_EINVAL, "NULL argument");
    struct Acc {
        long long n = 0;
        double ms = 0.0;
    };
    std::map<std::string, Acc> acc;
    for (auto &r : P->prof.recs) {
        HIP_OK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        std::string name(r.name);
        size_t a = name.find_first_not_of("( ");
        size_t b = name.find_first_of("<)", a);
        name = name.substr(a, b == std::string::npos ? std::string::npos : b - a);
        acc[name].n += 1;
        acc[name].ms += ms;
    }
    std::string out;
    for (auto &kv : acc) {
        char line[256];
        snprintf(line, sizeof(line), "%s %lld %.6f\n", kv.first.c_str(), kv.second.n, kv.second.ms);
        out += line;
    }
    std::snprintf(buf, len, "%s", out.c_str());
    return PFB_OK;
}

pfb_status pfb_grid(pfb_plan *P, const void *vis, void *image, int mode, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    const bool d = P->dbl;
    if (mode == PFB_GRID_DIRTY) {
        if (!vis || !image) return fail(PFB_EINVAL, "vis and image must be non-NULL");
        GridderHost &G = P->main;
        st = spread_prepass(P, 0, vis, s);
        if (st) return st;
        for (int b0 = 0; b0 < P->prob.n_band; b0 += P->band_batch) {
            const int nbb = std::min(P->band_batch, P->prob.n_band - b0);
            LAUNCH_OK(launch_spread(d, spread_args(P, G, b0, nbb, 0, vis, P->p(P->o_planes)), s));
            XformArgs xa = xform_args(P, G, b0, nbb);
            xa.image_out = image;
            LAUNCH_OK(launch_grid_xform(d, xa, s));
        }
        return PFB_OK;
    }
    if (mode == PFB_GRID_PSF) {
        GridderHost &G = P->psf;
        if (G.g.gx > (d ? 8192 : 16384) || G.g.gy > (d ? 8192 : 16384))
            return fail(PFB_EUNSUPPORTED, "the PSF of a %d x %d image needs FFT rows of %d points, longer than this "
                        "precision's %d", P->prob.nx, P->prob.ny, std::max(G.g.gx, G.g.gy), d ? 8192 : 16384);
        void *img = image ? image : P->p(P->o_psfimg);
        st = spread_prepass(P, 1, nullptr, s);
        if (st) return st;
        for (int b0 = 0; b0 < P->prob.n_band; b0 += P->band_batch) {
            const int nbb = std::min(P->band_batch, P->prob.n_band - b0);
            LAUNCH_OK(launch_spread(d, spread_args(P, G, b0, nbb, 1, nullptr, P->p(P->o_planes)), s));
            XformArgs xa = xform_args(P, G, b0, nbb);
            xa.image_out = img;
            xa.zero_edge = 1;
            LAUNCH_OK(launch_grid_xform(d, xa, s));
        }
        LAUNCH_OK(launch_psfhat(d, conv_args(P), img, s));
        P->psf_ready = true;
        return PFB_OK;
    }
    return fail(PFB_EINVAL, "unknown grid mode %d", mode);
}

pfb_status pfb_degrid(pfb_plan *P, const void *image, void *vis, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!image || !vis) return fail(PFB_EINVAL, "image and vis must be non-NULL");
    const bool d = P->dbl;
    GridderHost &G = P->main;
    LAUNCH_OK(launch_zero_flagged(d, reinterpret_cast<const uint32_t *>(P->p(P->o_flagged)), P->n_flagged, vis, s));
    for (int b0 = 0; b0 < P->prob.n_band; b0 += P->band_batch) {
        const int nbb = std::min(P->band_batch, P->prob.n_band - b0);
        XformArgs xa = xform_args(P, G, b0, nbb);
        xa.image_in = image;
        LAUNCH_OK(launch_degrid_xform(d, xa, s));
        LAUNCH_OK(launch_interp(d, interp_args(G, b0, nbb, 0, P->p(P->o_planes), vis), s));
    }
    return PFB_OK;
}

pfb_status pfb_degrid_add(pfb_plan *P, const void *image, void *vis, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!image || !vis) return fail(PFB_EINVAL, "image and vis must be non-NULL");
    const bool d = P->dbl;
    GridderHost &G = P->main;
    for (int b0 = 0; b0 < P->prob.n_band; b0 += P->band_batch) {
        const int nbb = std::min(P->band_batch, P->prob.n_band - b0);
        XformArgs xa = xform_args(P, G, b0, nbb);
        xa.image_in = image;
        LAUNCH_OK(launch_degrid_xform(d, xa, s));
        LAUNCH_OK(launch_interp(d, interp_args(G, b0, nbb, 2, P->p(P->o_planes), vis), s));
    }
    return PFB_OK;
}

pfb_status pfb_hessian(pfb_plan *P, const void *x, void *y, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!x || !y) return fail(PFB_EINVAL, "x and y must be non-NULL");
    if (x == y) return fail(PFB_EINVAL, "x and y must differ");
    return hessian_impl(P, x, y, s);
}

pfb_status pfb_psf_conv(pfb_plan *P, const void *x, void *y, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!x || !y) return fail(PFB_EINVAL, "x and y must be non-NULL");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    LAUNCH_OK(launch_psf_conv(P->dbl, conv_args(P), x, nullptr, y, nullptr, 0.0, CONV_IN_X, CONV_OUT_Y, s));
    return PFB_OK;
}

pfb_status pfb_precond_solve(pfb_plan *P, const void *g, void *y, double sigma, int iters, double tol,
                             double *dev_resid, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!g || !y) return fail(PFB_EINVAL, "g and y must be non-NULL");
    if (g == y) return fail(PFB_EINVAL, "g and y must differ");
    if (!(sigma >= 0) || !std::isfinite(sigma)) return fail(PFB_EINVAL, "sigma must be finite and >= 0");
    if (iters < 0) return fail(PFB_EINVAL, "iters must be >= 0");
    if (!(tol >= 0) || !std::isfinite(tol)) return fail(PFB_EINVAL, "tol must be finite and >= 0");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    if (tol > 0.0) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_OK(hipStreamIsCapturing(s, &cs));
        if (cs != hipStreamCaptureStatusNone)
            return fail(PFB_ESTATE, "tol > 0 reads the residual on the host and cannot be captured; use tol = 0");
    }
    st = cg_solve(P, g, y, sigma, iters, s, tol);
    if (st) return st;
    if (dev_resid) LAUNCH_OK(launch_copy_scalar(P->prob.n_band, reinterpret_cast<double *>(P->p(P->o_scal)), S_RR,
                                                dev_resid, s));
    return PFB_OK;
}

pfb_status pfb_power_iteration(pfb_plan *P, int op, const void *v0, int iters, double *dev_lambda, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!v0 || !dev_lambda) return fail(PFB_EINVAL, "v0 and dev_lambda must be non-NULL");
    if (op != 0 && op != 1) return fail(PFB_EINVAL, "op must be 0 (PSF) or 1 (Hessian)");
    if (iters < 0) return fail(PFB_EINVAL, "iters must be >= 0");
    if (op == 0 && !P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    const bool d = P->dbl;
    ConvArgs ca = conv_args(P);
    const int nb = P->prob.n_band;
    const int64_t Pn = (int64_t)P->prob.nx * P->prob.ny;
    char *v = reinterpret_cast<char *>(P->p(P->o_vec));
    void *wa = v + 3 * P->vec_bytes, *wb = v + 4 * P->vec_bytes, *tmp = v + 5 * P->vec_bytes;
    const int vparts = vec_partials_per_band(Pn);
    const int cparts = conv_partials_per_band(d, ca);
    const void *src = v0;
    LAUNCH_OK(launch_vec(d, VEC_NORM, nb, Pn, ca.partials, ca.max_partials, ca.scal, const_cast<void *>(src), nullptr,
                         nullptr, nullptr, nullptr, 0, 0, s));
    LAUNCH_OK(launch_reduce(RED_INV_SQRT, nb, ca.partials, vparts, ca.max_partials, ca.scal, s));
    for (int it = 0; it < iters; ++it) {
        void *dst = (it % 2 == 0) ? wa : wb;
        if (op == 0) {
            LAUNCH_OK(launch_psf_conv(d, ca, src, nullptr, dst, nullptr, 0.0, CONV_IN_SCALED, CONV_OUT_NORM, s));
            LAUNCH_OK(launch_reduce(RED_INV_SQRT, nb, ca.partials, cparts, ca.max_partials, ca.scal, s));
        } else {
            LAUNCH_OK(launch_vec(d, VEC_SCALE_COPY, nb, Pn, ca.partials, ca.max_partials, ca.scal,
                                 const_cast<void *>(src), tmp, nullptr, nullptr, nullptr, 0, 0, s));
            st = hessian_impl(P, tmp, dst, s);
            if (st) return st;
            LAUNCH_OK(launch_vec(d, VEC_NORM, nb, Pn, ca.partials, ca.max_partials, ca.scal, dst, nullptr, nullptr,
                                 nullptr, nullptr, 0, 0, s));
            LAUNCH_OK(launch_reduce(RED_INV_SQRT, nb, ca.partials, vparts, ca.max_partials, ca.scal, s));
        }
        src = dst;
    }
    // lambda = v^T A v with v = src * scale
    void *dst = (iters % 2 == 0) ? wa : wb;
    LAUNCH_OK(launch_vec(d, VEC_SCALE_COPY, nb, Pn, ca.partials, ca.max_partials, ca.scal, const_cast<void *>(src), tmp,
                         nullptr, nullptr, nullptr, 0, 0, s));
    if (op == 0) {
        LAUNCH_OK(launch_psf_conv(d, ca, tmp, nullptr, dst, tmp, 0.0, CONV_IN_X, CONV_OUT_DOT, s));
        LAUNCH_OK(launch_reduce(RED_LAMBDA, nb, ca.partials, cparts, ca.max_partials, ca.scal, s));
    } else {
        st = hessian_impl(P, tmp, dst, s);
        if (st) return st;
        LAUNCH_OK(launch_vec(d, VEC_DOT, nb, Pn, ca.partials, ca.max_partials, ca.scal, tmp, dst, nullptr, nullptr,
                             nullptr, 0, 0, s));
        LAUNCH_OK(launch_reduce(RED_LAMBDA, nb, ca.partials, vparts, ca.max_partials, ca.scal, s));
    }
    LAUNCH_OK(launch_copy_scalar(nb, ca.scal, S_LAMBDA, dev_lambda, s));
    return PFB_OK;
}

pfb_status pfb_fb_step(pfb_plan *P, const void *dirty, void *x, double sigma, double gamma, double lambda,
                       int cg_iters, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!dirty || !x) return fail(PFB_EINVAL, "dirty and x must be non-NULL");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    if (!(sigma >= 0) || !(gamma > 0) || !(lambda >= 0) || cg_iters < 0)
        return fail(PFB_EINVAL, "need sigma >= 0, gamma > 0, lambda >= 0, cg_iters >= 0");
    const bool d = P->dbl;
    ConvArgs ca = conv_args(P);
    char *v = reinterpret_cast<char *>(P->p(P->o_vec));
    void *g = v + 3 * P->vec_bytes, *y = v + 4 * P->vec_bytes;
    LAUNCH_OK(launch_psf_conv(d, ca, x, nullptr, g, dirty, 0.0, CONV_IN_X, CONV_OUT_SUB, s));
    st = cg_solve(P, g, y, sigma, cg_iters, s);
    if (st) return st;
    const int64_t Pn = (int64_t)P->prob.nx * P->prob.ny;
    LAUNCH_OK(launch_vec(d, VEC_FB_PROX, P->prob.n_band, Pn, ca.partials, ca.max_partials, ca.scal, x, y, nullptr,
                         nullptr, nullptr, gamma, lambda, s));
    return PFB_OK;
}


// ---------------------------------------------------------------------------
// backward step (eq. 7 with the regulariser of eq. 9)
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr int kMaxBases = 7;   // Dirac + db1 .. db6

// Low-pass filter of the Daubechies wavelet with n vanishing moments (length 2n):
// |m0|^2 = cos^(2n)(xi/2) P(sin^2(xi/2)), P(y) = sum_{k<n} C(n-1+k, k) y^k.  The
// roots of P (Durand-Kerner iteration) map to z-plane pairs z + 1/z = 2 - 4y; the
// filter polynomial (z + 1)^n prod (z - z_i) takes the root inside the unit circle
// (minimum phase); h lists its coefficients in descending powers, scaled to sum
// sqrt(2).
void daubechies_filter(int n, double *h) {
    using C = std::complex<double>;
    const int deg = n - 1;
    std::vector<double> a(n);
    for (int k = 0; k < n; ++k) {
        double c = 1.0;
        for (int i = 1; i <= k; ++i) c = c * (double)(n - 1 + i) / (double)i;
        a[k] = c;
    }
    std::vector<C> y(deg);
    for (int i = 0; i < deg; ++i) y[i] = std::pow(C(0.4, 0.9), i);
    auto poly_at = [&](C t) {
        C r = a[deg];
        for (int k = deg - 1; k >= 0; --k) r = r * t + a[k];
        return r;
    };
    for (int it = 0; it < 1000 && deg > 0; ++it) {
        double moved = 0.0;
        for (int i = 0; i < deg; ++i) {
            C den = a[deg];
            for (int j = 0; j < deg; ++j)
                if (j != i) den *= (y[i] - y[j]);
            const C step = poly_at(y[i]) / den;
            y[i] -= step;
            moved = std::max(moved, std::abs(step) / std::max(1.0, std::abs(y[i])));
        }
        if (moved < 1e-15) break;
    }
    std::vector<C> roots(n, C(-1.0, 0.0));
    for (const C &yy : y) {
        const C b = 1.0 - 2.0 * yy;
        const C sq = std::sqrt(b * b - 1.0);
        const C z1 = b + sq, z2 = b - sq;
        roots.push_back(std::abs(z1) < 1.0 ? z1 : z2);
    }
    std::vector<C> poly{C(1.0, 0.0)};
    for (const C &r : roots) {
        std::vector<C> next(poly.size() + 1, C(0.0, 0.0));
        for (size_t i = 0; i < poly.size(); ++i) {
            next[i] += poly[i];
            next[i + 1] -= r * poly[i];
        }
        poly.swap(next);
    }
    double sum = 0.0;
    for (int i = 0; i < 2 * n; ++i) {
        h[i] = poly[i].real();
        sum += h[i];
    }
    for (int i = 0; i < 2 * n; ++i) h[i] *= std::sqrt(2.0) / sum;
}

// db1 .. db6, computed once per process (the initialisation of a function-local
// static is thread-safe)
WaveletFilter db_filter(int n) {
    static const std::vector<WaveletFilter> table = [] {
        std::vector<WaveletFilter> t(kMaxBases);
        for (int k = 1; k < kMaxBases; ++k) {
            t[k].len = 2 * k;
            daubechies_filter(k, t[k].h);
        }
        return t;
    }();
    return table[n];
}

// element offsets (in reals) of the prox workspace: v, coef, then six image buffers
struct ProxLayout {
    int64_t NP;          // n_band * nx * ny
    size_t v, coef, d, c, u, sv, a, b, z, total;   // bytes
};
ProxLayout prox_layout(const pfb_plan *P, int nbasis) {
    ProxLayout L{};
    L.NP = (int64_t)P->prob.n_band * P->prob.nx * P->prob.ny;
    const size_t img = (size_t)L.NP * P->rsz;
    L.v = 0;
    L.coef = L.v + (size_t)nbasis * img;
    L.d = L.coef + (size_t)(nbasis - 1) * img;
    L.c = L.d + img;
    L.u = L.c + img;
    L.sv = L.u + img;
    L.a = L.sv + img;
    L.b = L.a + img;
    L.z = L.b + img;      // forward-step result of pfb_fb_step_wavelet
    L.total = L.z + img;
    return L;
}

pfb_status wavelet_args_ok(const pfb_plan *P, int nbasis, int levels) {
    if (nbasis < 1 || nbasis > kMaxBases) return fail(PFB_EINVAL, "nbasis must be 1 .. %d", kMaxBases);
    if (levels < 1 || levels > 16) return fail(PFB_EINVAL, "levels must be 1 .. 16");
    const int m = (1 << levels) - 1;
    if ((P->prob.nx & m) || (P->prob.ny & m))
        return fail(PFB_EINVAL, "nx = %d and ny = %d must be multiples of 2^levels = %d", P->prob.nx, P->prob.ny,
                    1 << levels);
    return PFB_OK;
}

// coef_k (k >= 1) = W_k^dagger src for every band, unscaled; the low-pass block
// of every level but the last goes to buffer a or b (alternately)
pfb_status analysis_bases(const pfb_plan *P, const void *src, char *coef, void *a, void *b, int nbasis, int levels,
                          hipStream_t s) {
    const bool d = P->dbl;
    const int nx = P->prob.nx, ny = P->prob.ny, nb = P->prob.n_band;
    const int64_t Pn = (int64_t)nx * ny;
    const size_t img = (size_t)nb * Pn * P->rsz;
    void *pp[2] = {a, b};
    for (int k = 1; k < nbasis; ++k) {
        const WaveletFilter f = db_filter(k);
        void *ck = coef + (size_t)(k - 1) * img;
        for (int l = 0; l < levels; ++l) {
            const void *in = l == 0 ? src : pp[(l - 1) & 1];
            void *ll = l == levels - 1 ? ck : pp[l & 1];
            LAUNCH_OK(launch_wavelet_analysis_level(d, in, ck, ll, f, nx >> l, ny >> l, ny, Pn, nb, s));
        }
    }
    return PFB_OK;
}

// out = v_0 + sum_{k >= 1} W_k v_k (unscaled); the low-pass block of every level
// but the finest goes to buffer a or b (alternately)
pfb_status synthesis_bases(const pfb_plan *P, const char *v, void *out, void *a, void *b, int nbasis, int levels,
                           hipStream_t s) {
    const bool d = P->dbl;
    const int nx = P->prob.nx, ny = P->prob.ny, nb = P->prob.n_band;
    const int64_t Pn = (int64_t)nx * ny;
    const size_t img = (size_t)nb * Pn * P->rsz;
    void *pp[2] = {a, b};
    LAUNCH_OK(launch_wave_copy(d, v, out, (int64_t)nb * Pn, 1.0, s));
    for (int k = 1; k < nbasis; ++k) {
        const WaveletFilter f = db_filter(k);
        const void *vk = v + (size_t)k * img;
        for (int l = levels - 1; l >= 0; --l) {
            const void *ll = l == levels - 1 ? vk : pp[(l + 1) & 1];
            void *dst = l == 0 ? out : pp[l & 1];
            LAUNCH_OK(launch_wavelet_synthesis_level(d, l == 0, ll, vk, dst, f, nx >> l, ny >> l, ny, Pn, nb, s));
        }
    }
    return PFB_OK;
}

}  // namespace

extern "C" {

pfb_status pfb_prox_workspace_size(const pfb_plan *P, int nbasis, size_t *bytes) {
    if (!P || !bytes) return fail(PFB_EINVAL, "plan and bytes must be non-NULL");
    if (nbasis < 1 || nbasis > kMaxBases) return fail(PFB_EINVAL, "nbasis must be 1 .. %d", kMaxBases);
    *bytes = prox_layout(P, nbasis).total;
    return PFB_OK;
}

pfb_status pfb_wavelet_analysis(pfb_plan *P, const void *x, void *coeffs, void *ws, size_t ws_bytes, int nbasis,
                                int levels, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!x || !coeffs || !ws) return fail(PFB_EINVAL, "x, coeffs and ws must be non-NULL");
    if ((st = wavelet_args_ok(P, nbasis, levels))) return st;
    const ProxLayout L = prox_layout(P, nbasis);
    if (ws_bytes < L.total) return fail(PFB_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    const bool d = P->dbl;
    const double scale = 1.0 / std::sqrt((double)nbasis);
    char *c = reinterpret_cast<char *>(coeffs);
    char *w = reinterpret_cast<char *>(ws);
    const size_t img = (size_t)L.NP * P->rsz;
    LAUNCH_OK(launch_wave_copy(d, x, c, L.NP, scale, s));
    if ((st = analysis_bases(P, x, c + img, w + L.a, w + L.b, nbasis, levels, s))) return st;
    if (nbasis > 1) LAUNCH_OK(launch_wave_copy(d, c + img, c + img, (int64_t)(nbasis - 1) * L.NP, scale, s));
    return PFB_OK;
}

pfb_status pfb_wavelet_synthesis(pfb_plan *P, const void *coeffs, void *x, void *ws, size_t ws_bytes, int nbasis,
                                 int levels, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!x || !coeffs || !ws) return fail(PFB_EINVAL, "coeffs, x and ws must be non-NULL");
    if ((st = wavelet_args_ok(P, nbasis, levels))) return st;
    const ProxLayout L = prox_layout(P, nbasis);
    if (ws_bytes < L.total) return fail(PFB_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    char *w = reinterpret_cast<char *>(ws);
    if ((st = synthesis_bases(P, reinterpret_cast<const char *>(coeffs), x, w + L.a, w + L.b, nbasis, levels, s)))
        return st;
    LAUNCH_OK(launch_wave_copy(P->dbl, x, x, L.NP, 1.0 / std::sqrt((double)nbasis), s));
    return PFB_OK;
}

pfb_status pfb_prox_solve(pfb_plan *P, const void *z, void *x, void *ws, size_t ws_bytes, int nbasis, int levels,
                          double lambda, double gamma, double sigma, double unorm, int iters, int warm,
                          hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!z || !x || !ws) return fail(PFB_EINVAL, "z, x and ws must be non-NULL");
    if (z == x) return fail(PFB_EINVAL, "z and x must differ");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    if ((st = wavelet_args_ok(P, nbasis, levels))) return st;
    if (!(lambda >= 0) || !(gamma > 0) || !(sigma >= 0) || !(unorm > 0) || !std::isfinite(lambda) ||
        !std::isfinite(gamma) || !std::isfinite(sigma) || !std::isfinite(unorm) || iters < 0)
        return fail(PFB_EINVAL, "need lambda >= 0, gamma > 0, sigma >= 0, unorm > 0 (finite), iters >= 0");
    const ProxLayout L = prox_layout(P, nbasis);
    if (ws_bytes < L.total) return fail(PFB_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    const bool d = P->dbl;
    char *w = reinterpret_cast<char *>(ws);
    void *v = w + L.v, *coef = w + L.coef, *dd = w + L.d, *c = w + L.c, *u = w + L.u, *sv = w + L.sv;
    // Condat's iteration: F(x) = (x - z)^T U (x - z) / (2 gamma) with U = I^psf * + sigma Id,
    // G = positivity, H = lambda ||.||_{2,1} of L x = Psi^dagger x (||Psi^dagger|| = 1)
    const double beta = (unorm + sigma) / gamma;
    const double sigma_d = beta, tau = 0.99 / (0.5 * beta + sigma_d);
    const double psi_scale = 1.0 / std::sqrt((double)nbasis);
    const ConvArgs ca = conv_args(P);
    if (!warm) LAUNCH_OK(launch_pd_dual(d, true, v, nullptr, nullptr, nbasis, P->prob.n_band,
                                         (int64_t)P->prob.nx * P->prob.ny, 0.0, 0.0, 0.0, s));
    LAUNCH_OK(launch_pd_primal(d, true, z, x, dd, nullptr, nullptr, nullptr, L.NP, 0.0, 1.0, 0.0, 0.0, warm, s));
    for (int it = 0; it < iters; ++it) {
        LAUNCH_OK(launch_psf_conv(d, ca, dd, nullptr, c, nullptr, 0.0, CONV_IN_X, CONV_OUT_Y, s));
        if ((st = synthesis_bases(P, reinterpret_cast<const char *>(v), sv, w + L.a, w + L.b, nbasis, levels, s)))
            return st;
        LAUNCH_OK(launch_pd_primal(d, false, z, x, dd, c, sv, u, L.NP, tau, gamma, sigma, psi_scale, warm, s));
        if ((st = analysis_bases(P, u, reinterpret_cast<char *>(coef), w + L.a, w + L.b, nbasis, levels, s))) return st;
        LAUNCH_OK(launch_pd_dual(d, false, v, u, coef, nbasis, P->prob.n_band, (int64_t)P->prob.nx * P->prob.ny,
                                 sigma_d, psi_scale, lambda, s));
    }
    return PFB_OK;
}

pfb_status pfb_fb_step_wavelet(pfb_plan *P, const void *dirty, void *x, void *ws, size_t ws_bytes, int nbasis,
                               int levels, double sigma, double gamma, double lambda, double unorm, int cg_iters,
                               int pd_iters, int warm, hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!dirty || !x || !ws) return fail(PFB_EINVAL, "dirty, x and ws must be non-NULL");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    if ((st = wavelet_args_ok(P, nbasis, levels))) return st;
    if (!(sigma >= 0) || !(gamma > 0) || cg_iters < 0) return fail(PFB_EINVAL, "need sigma >= 0, gamma > 0, cg_iters >= 0");
    const ProxLayout L = prox_layout(P, nbasis);
    if (ws_bytes < L.total) return fail(PFB_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    const bool d = P->dbl;
    ConvArgs ca = conv_args(P);
    char *v = reinterpret_cast<char *>(P->p(P->o_vec));
    void *g = v + 3 * P->vec_bytes, *y = v + 4 * P->vec_bytes;
    void *z = reinterpret_cast<char *>(ws) + L.z;
    // forward step (eq. 6): z = x - gamma U^-1 (I^psf * x - I^d)
    LAUNCH_OK(launch_psf_conv(d, ca, x, nullptr, g, dirty, 0.0, CONV_IN_X, CONV_OUT_SUB, s));
    st = cg_solve(P, g, y, sigma, cg_iters, s);
    if (st) return st;
    LAUNCH_OK(launch_wave_axpy(d, x, y, z, L.NP, -gamma, s));
    // backward step (eq. 7 with the regulariser of eq. 9)
    return pfb_prox_solve(P, z, x, ws, ws_bytes, nbasis, levels, lambda, gamma, sigma, unorm, pd_iters, warm, s);
}

pfb_status pfb_clean(pfb_plan *P, const void *dirty, void *x, void *ws, size_t ws_bytes, int nbasis, int levels,
                     double sigma, double gamma, double lambda, double unorm, int cg_iters, int pd_iters, int n_major,
                     hipStream_t s) {
    ProfScope prof_scope(P);
    pfb_status st = check_ready(P);
    if (st) return st;
    if (!dirty || !x || !ws) return fail(PFB_EINVAL, "dirty, x and ws must be non-NULL");
    if (!P->psf_ready) return fail(PFB_ESTATE, "no PSF spectrum: call pfb_grid with PFB_GRID_PSF first");
    if ((st = wavelet_args_ok(P, nbasis, levels))) return st;
    if (!(sigma >= 0) || !(gamma > 0) || cg_iters < 0 || n_major < 0)
        return fail(PFB_EINVAL, "need sigma >= 0, gamma > 0, cg_iters >= 0, n_major >= 0");
    const ProxLayout L = prox_layout(P, nbasis);
    if (ws_bytes < L.total) return fail(PFB_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    const bool d = P->dbl;
    char *v = reinterpret_cast<char *>(P->p(P->o_vec));
    void *g = v + 3 * P->vec_bytes, *y = v + 4 * P->vec_bytes;
    void *z = reinterpret_cast<char *>(ws) + L.z;
    for (int k = 0; k < n_major; ++k) {
        // exact gradient (eq. 3): R^dagger Sigma^-1 R x - I^d, one Hessian application
        if ((st = hessian_impl(P, x, g, s))) return st;
        LAUNCH_OK(launch_wave_axpy(d, g, dirty, g, L.NP, -1.0, s));
        // forward step (eq. 6) preconditioned by U = I^psf * + sigma Id, backward step (eq. 7)
        if ((st = cg_solve(P, g, y, sigma, cg_iters, s))) return st;
        LAUNCH_OK(launch_wave_axpy(d, x, y, z, L.NP, -gamma, s));
        if ((st = pfb_prox_solve(P, z, x, ws, ws_bytes, nbasis, levels, lambda, gamma, sigma, unorm, pd_iters, k > 0,
                                 s)))
            return st;
    }
    return PFB_OK;
}

}  // extern "C"
