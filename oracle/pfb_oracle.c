/*
 * FP64 direct-sum reference for the radio-interferometric measurement operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; it exists so that the tests, the smoke check and the
 * CPU-baseline leg of the benchmark have an independent, obviously-correct
 * answer to compare with.  It shares no code with the HIP path.
 *
 * What it computes (Bester et al., "A practical preconditioner for wide-field
 * continuum imaging of radio interferometric data", Section 2):
 *   - the measurement model V = R x + eps with diagonal Sigma (eq. 1);
 *     R maps n_b real images of n_p pixels to n_nu x n_d complex visibilities,
 *     one band per group of channels;
 *   - R itself is written out as the plain direct sum that the paper's 2-D
 *     NUFFT with wide-field correction approximates:
 *         V_rc = sum_p x_{b(c)}[p] exp(-2 pi i (u l_p + v m_p + w (n_p - 1))) / n_p
 *     with (u, v, w) = uvw_r * f_c / c0 in wavelengths;
 *   - the dirty image I^d = R^dagger Sigma^-1 V (Section 2, after eq. 3), the
 *     real part of the weighted adjoint sum;
 *   - the point spread function used by the approximate gradient (eq. 4), in
 *     its flat form (no w term, n = 1) on a 2nx x 2ny grid: the dirty image of
 *     unit visibilities.
 *
 * Conventions (the paper is silent on them; the readings are listed in the
 * design notes): pixel (i, j) sits at l = (i - nx/2) cellx, m = (j - ny/2)
 * celly, axis 0 is l; n - 1 is evaluated as -(l^2 + m^2) / (1 + n) to avoid
 * cancellation; the phase in cycles is reduced by its nearest integer before
 * sin/cos.  Sums use Neumaier compensation so that the oracle's own rounding
 * stays far below the 1e-10 relative tolerance of the FP64 comparison.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define C0 299792458.0
#define TWO_PI 6.283185307179586476925286766559

typedef struct { double s, c; } ksum;   /* Neumaier running sum and compensation */

static inline void kadd(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else                       k->c += (x - t) + k->s;
    k->s = t;
}
static inline double kval(const ksum *k) { return k->s + k->c; }

/* direction cosines of pixel (i, j) of an nx x ny grid and n - 1, n */
static inline void pixel_lmn(int64_t i, int64_t j, int nx, int ny, double cellx, double celly,
                             double *l, double *m, double *nm1, double *n)
{
    double L = (double)(i - nx / 2) * cellx;
    double M = (double)(j - ny / 2) * celly;
    double r2 = L * L + M * M;
    double N = sqrt(1.0 - r2);
    *l = L; *m = M; *n = N;
    *nm1 = -r2 / (1.0 + N);
}

/* cos and sin of 2 pi t with t in cycles, after removing the nearest integer */
static inline void cis_cycles(double t, double *c, double *s)
{
    double f = t - nearbyint(t);
    *c = cos(TWO_PI * f);
    *s = sin(TWO_PI * f);
}

/*
 * Degrid: V for the selected visibilities.
 *   sel[k] = r * n_chan + c          (n_sel entries)
 *   the image is given as a sparse list of pixels: pix[q] = b*nx*ny + i*ny + j,
 *   val[q] its value (a dense image is simply every pixel)
 *   weight is diag(Sigma^-1) with flagged entries already zero; V = 0 there.
 *   flat != 0 drops the w term and the 1/n factor.
 * out[2k], out[2k+1] = Re, Im of V.
 */
void oracle_degrid(int64_t n_row, int64_t n_chan, const int32_t *chan_band,
                   const double *freq, const double *uvw, const double *weight,
                   int nx, int ny, double cellx, double celly, int flat,
                   int64_t n_pix, const int64_t *pix, const double *val,
                   int64_t n_sel, const int64_t *sel, double *out)
{
    (void)n_row;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_sel; ++k) {
        int64_t rc = sel[k];
        int64_t r = rc / n_chan, c = rc % n_chan;
        if (weight[rc] == 0.0) { out[2 * k] = 0.0; out[2 * k + 1] = 0.0; continue; }
        double s = freq[c] / C0;
        double u = uvw[3 * r] * s, v = uvw[3 * r + 1] * s, w = uvw[3 * r + 2] * s;
        int b = chan_band[c];
        ksum re = {0, 0}, im = {0, 0};
        for (int64_t q = 0; q < n_pix; ++q) {
            int64_t p = pix[q];
            int64_t pb = p / ((int64_t)nx * ny);
            if (pb != b) continue;
            int64_t pij = p % ((int64_t)nx * ny);
            double l, m, nm1, n;
            pixel_lmn(pij / ny, pij % ny, nx, ny, cellx, celly, &l, &m, &nm1, &n);
            double t = u * l + v * m + (flat ? 0.0 : w * nm1);
            double cs, sn;
            cis_cycles(t, &cs, &sn);
            double a = val[q] / (flat ? 1.0 : n);
            /* exp(-2 pi i t) = cos - i sin */
            kadd(&re, a * cs);
            kadd(&im, -a * sn);
        }
        out[2 * k] = kval(&re);
        out[2 * k + 1] = kval(&im);
    }
}

/*
 * Grid (weighted adjoint): I_b[p] = Re sum_{r, c in b} w_rc V_rc exp(+2 pi i t) / n_p
 * for the selected pixels pix[q] = b*nx*ny + i*ny + j.  vis is [n_row][n_chan][2].
 */
void oracle_grid(int64_t n_row, int64_t n_chan, const int32_t *chan_band,
                 const double *freq, const double *uvw, const double *weight,
                 int nx, int ny, double cellx, double celly, int flat,
                 const double *vis, int64_t n_pix, const int64_t *pix, double *out)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t p = pix[q];
        int64_t b = p / ((int64_t)nx * ny);
        int64_t pij = p % ((int64_t)nx * ny);
        double l, m, nm1, n;
        pixel_lmn(pij / ny, pij % ny, nx, ny, cellx, celly, &l, &m, &nm1, &n);
        ksum acc = {0, 0};
        for (int64_t r = 0; r < n_row; ++r) {
            for (int64_t c = 0; c < n_chan; ++c) {
                if (chan_band[c] != b) continue;
                int64_t rc = r * n_chan + c;
                double wt = weight[rc];
                if (wt == 0.0) continue;
                double s = freq[c] / C0;
                double u = uvw[3 * r] * s, v = uvw[3 * r + 1] * s, w = uvw[3 * r + 2] * s;
                double t = u * l + v * m + (flat ? 0.0 : w * nm1);
                double cs, sn;
                cis_cycles(t, &cs, &sn);
                /* Re[(Vr + i Vi)(cos + i sin)] = Vr cos - Vi sin */
                kadd(&acc, wt * (vis[2 * rc] * cs - vis[2 * rc + 1] * sn));
            }
        }
        out[q] = kval(&acc) / (flat ? 1.0 : n);
    }
}

/*
 * Flat PSF on the 2nx x 2ny grid: pixel (i', j') is offset (i' - nx, j' - ny)
 * cells from the centre; PSF = sum w cos(2 pi (u dl + v dm)).  Row 0 and
 * column 0 (offset -nx / -ny) are set to zero.  pix[q] = b*(2nx)(2ny) + i'*(2ny) + j'.
 */
void oracle_psf(int64_t n_row, int64_t n_chan, const int32_t *chan_band,
                const double *freq, const double *uvw, const double *weight,
                int nx, int ny, double cellx, double celly,
                int64_t n_pix, const int64_t *pix, double *out)
{
    int64_t NX = 2 * (int64_t)nx, NY = 2 * (int64_t)ny;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t p = pix[q];
        int64_t b = p / (NX * NY);
        int64_t ip = (p % (NX * NY)) / NY, jp = p % NY;
        if (ip == 0 || jp == 0) { out[q] = 0.0; continue; }
        double dl = (double)(ip - nx) * cellx, dm = (double)(jp - ny) * celly;
        ksum acc = {0, 0};
        for (int64_t r = 0; r < n_row; ++r) {
            for (int64_t c = 0; c < n_chan; ++c) {
                if (chan_band[c] != b) continue;
                int64_t rc = r * n_chan + c;
                double wt = weight[rc];
                if (wt == 0.0) continue;
                double s = freq[c] / C0;
                double cs, sn;
                cis_cycles(uvw[3 * r] * s * dl + uvw[3 * r + 1] * s * dm, &cs, &sn);
                kadd(&acc, wt * cs);
            }
        }
        out[q] = kval(&acc);
    }
}

/* number of OpenMP threads the oracle runs with (reported by the benchmark) */
int oracle_threads(void)
{
    int n = 1;
    #pragma omp parallel
    {
        #pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
