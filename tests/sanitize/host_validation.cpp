// Sanitizer driver for the library's host code (test infrastructure): built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side by
// tests/test_sanitize.py and linked with the library's objects.  It runs the
// argument and shape validation that needs no GPU (null arguments, odd or too
// small sides, bad bands, bad options, epsilon, facet offsets) and checks the
// documented status codes.  Exits 0 when every check passes.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "pfb.h"

static int fails = 0;
static void expect(bool ok, const char *what) {
    if (!ok) {
        std::printf("FAILED: %s (last error: %s)\n", what, pfb_last_error());
        ++fails;
    }
}

int main() {
    expect(std::strstr(pfb_version(), "gfx950") != nullptr, "version names gfx950");
    pfb_plan *h = nullptr;
    expect(pfb_plan_create(nullptr, nullptr, nullptr, nullptr) == PFB_EINVAL, "null plan pointer");
    expect(pfb_plan_create(&h, nullptr, nullptr, nullptr) == PFB_EINVAL, "null problem");
    expect(pfb_plan_destroy(nullptr) == PFB_OK, "destroy null");
    double freq[2] = {1e9, 1.1e9};
    int32_t cb[2] = {0, 0};
    pfb_problem prob;
    std::memset(&prob, 0, sizeof prob);
    prob.n_row = 10;
    prob.n_chan = 2;
    prob.n_band = 1;
    prob.chan_band = cb;
    prob.freq = freq;
    prob.uvw = reinterpret_cast<const double *>(16);   // never dereferenced: validation fails first
    prob.weight = reinterpret_cast<const void *>(16);
    prob.nx = 25;
    prob.ny = 32;
    prob.cellx = prob.celly = 1e-4;
    pfb_options opt;
    std::memset(&opt, 0, sizeof opt);
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EINVAL, "odd side");
    prob.nx = 14;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EINVAL, "side below 16");
    prob.nx = 32;
    opt.support = 3;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EINVAL, "support 3");
    opt.support = 0;
    opt.tile = 48;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EINVAL, "tile not a power of two");
    opt.tile = 0;
    for (double bad : {-1e-3, (double)std::nan(""), (double)INFINITY, 1e-9}) {
        opt.epsilon = bad;
        expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EINVAL, "bad epsilon");
    }
    opt.epsilon = 0.0;
    prob.nx = prob.ny = 8192;
    prob.cellx = prob.celly = 1e-7;
    opt.precision = 1;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EUNSUPPORTED, "FP64 rows too long");
    opt.precision = 0;
    prob.nx = prob.ny = 256;
    prob.cellx = prob.celly = 1e-4;
    cb[1] = 3;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EINVAL, "chan_band out of range");
    cb[1] = 0;
    prob.offx = 3;
    opt.precision = 1;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EUNSUPPORTED, "facet offset in FP64");
    opt.precision = 0;
    opt.flat = 1;
    expect(pfb_plan_create(&h, &prob, &opt, nullptr) == PFB_EUNSUPPORTED, "facet offset in flat mode");
    size_t n = 0;
    expect(pfb_plan_count_scratch_size(nullptr, &n) == PFB_EINVAL, "count scratch size without plan");
    expect(pfb_precond_solve(nullptr, nullptr, nullptr, 1.0, 1, 0.0, nullptr, nullptr) == PFB_EINVAL, "solve without plan");
    std::printf(fails ? "FAILED\n" : "ok\n");
    return fails ? 1 : 0;
}
