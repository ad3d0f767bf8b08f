/*
 * Sanitizer driver for the C oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize.py and
 * run on a small seeded problem.  Besides the sanitizers' own checks it tests
 * properties of the direct sums that hold exactly (up to rounding):
 *   - the weighted adjoint identity <R x, W y> = <x, R^dagger W y> (eq. 1 and
 *     the dirty image after eq. 3), w-term on and off;
 *   - the flat PSF (eq. 4) is symmetric about its centre and peaks at the sum
 *     of the band's weights, with row 0 and column 0 zero.
 * Exits 0 when every check passes.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_degrid(int64_t n_row, int64_t n_chan, const int32_t *chan_band, const double *freq,
                   const double *uvw, const double *weight, int nx, int ny, double cellx, double celly,
                   int flat, int64_t n_pix, const int64_t *pix, const double *val, int64_t n_sel,
                   const int64_t *sel, double *out);
void oracle_grid(int64_t n_row, int64_t n_chan, const int32_t *chan_band, const double *freq,
                 const double *uvw, const double *weight, int nx, int ny, double cellx, double celly,
                 int flat, const double *vis, int64_t n_pix, const int64_t *pix, double *out);
void oracle_psf(int64_t n_row, int64_t n_chan, const int32_t *chan_band, const double *freq,
                const double *uvw, const double *weight, int nx, int ny, double cellx, double celly,
                int64_t n_pix, const int64_t *pix, double *out);

static uint64_t state = 0x2101080722ULL;
static double urand(void) {   /* 64-bit LCG (Knuth's MMIX constants), top 53 bits */
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    enum { NROW = 40, NCHAN = 3, NX = 12, NY = 10, NB = 2 };
    const int32_t chan_band[NCHAN] = {0, 0, 1};
    const double freq[NCHAN] = {1.0e9, 1.1e9, 1.2e9};
    const double cell = 2.0e-3;   /* radians: |l|, |m| up to 0.012, n - 1 ~ -7e-5 */
    double *uvw = malloc(sizeof(double) * 3 * NROW);
    double *wt = malloc(sizeof(double) * NROW * NCHAN);
    double *x = malloc(sizeof(double) * NB * NX * NY);
    double *y = malloc(sizeof(double) * 2 * NROW * NCHAN);
    double *rx = malloc(sizeof(double) * 2 * NROW * NCHAN);
    double *gy = malloc(sizeof(double) * NB * NX * NY);
    int64_t *pix = malloc(sizeof(int64_t) * NB * NX * NY);
    int64_t *sel = malloc(sizeof(int64_t) * NROW * NCHAN);
    const int64_t npsf = (int64_t)NB * 4 * NX * NY;
    int64_t *ppix = malloc(sizeof(int64_t) * npsf);
    double *psf = malloc(sizeof(double) * npsf);
    for (int r = 0; r < NROW; ++r)
        for (int k = 0; k < 3; ++k) uvw[3 * r + k] = (urand() - 0.5) * (k == 2 ? 400.0 : 2000.0);
    for (int e = 0; e < NROW * NCHAN; ++e) wt[e] = urand() < 0.1 ? 0.0 : 0.5 + urand();
    for (int p = 0; p < NB * NX * NY; ++p) { x[p] = urand() - 0.5; pix[p] = p; }
    for (int e = 0; e < NROW * NCHAN; ++e) { y[2 * e] = urand() - 0.5; y[2 * e + 1] = urand() - 0.5; sel[e] = e; }
    int fails = 0;
    for (int flat = 0; flat < 2; ++flat) {
        oracle_degrid(NROW, NCHAN, chan_band, freq, uvw, wt, NX, NY, cell, cell, flat, NB * NX * NY, pix, x,
                      NROW * NCHAN, sel, rx);
        oracle_grid(NROW, NCHAN, chan_band, freq, uvw, wt, NX, NY, cell, cell, flat, y, NB * NX * NY, pix, gy);
        double lhs = 0.0, rhs = 0.0, scale = 0.0;
        for (int e = 0; e < NROW * NCHAN; ++e) {
            lhs += wt[e] * (rx[2 * e] * y[2 * e] + rx[2 * e + 1] * y[2 * e + 1]);
            scale += wt[e] * (fabs(rx[2 * e] * y[2 * e]) + fabs(rx[2 * e + 1] * y[2 * e + 1]));
        }
        for (int p = 0; p < NB * NX * NY; ++p) rhs += x[p] * gy[p];
        const double err = fabs(lhs - rhs) / scale;
        printf("adjoint (flat=%d): <Rx, Wy> = %.15g, <x, R'Wy> = %.15g, rel %.2e\n", flat, lhs, rhs, err);
        if (!(err < 1e-12)) ++fails;
    }
    for (int64_t q = 0; q < npsf; ++q) ppix[q] = q;
    oracle_psf(NROW, NCHAN, chan_band, freq, uvw, wt, NX, NY, cell, cell, npsf, ppix, psf);
    for (int b = 0; b < NB; ++b) {
        const double *P = psf + (int64_t)b * 4 * NX * NY;
        double sw = 0.0, asym = 0.0;
        for (int r = 0; r < NROW; ++r)
            for (int c = 0; c < NCHAN; ++c)
                if (chan_band[c] == b) sw += wt[r * NCHAN + c];
        for (int i = 1; i < 2 * NX; ++i)
            for (int j = 1; j < 2 * NY; ++j)
                asym = fmax(asym, fabs(P[i * 2 * NY + j] - P[(2 * NX - i) * 2 * NY + (2 * NY - j)]));
        double edge = 0.0;
        for (int i = 0; i < 2 * NX; ++i) edge = fmax(edge, fabs(P[i * 2 * NY]));
        for (int j = 0; j < 2 * NY; ++j) edge = fmax(edge, fabs(P[j]));
        const double peak = P[NX * 2 * NY + NY];
        printf("psf band %d: peak %.15g (sum of weights %.15g), max asymmetry %.2e, edge %.1e\n", b, peak, sw, asym, edge);
        if (!(fabs(peak - sw) <= 1e-12 * sw && asym <= 1e-12 * sw && edge == 0.0)) ++fails;
    }
    free(uvw); free(wt); free(x); free(y); free(rx); free(gy); free(pix); free(sel); free(ppix); free(psf);
    printf(fails ? "FAILED\n" : "ok\n");
    return fails ? 1 : 0;
}
