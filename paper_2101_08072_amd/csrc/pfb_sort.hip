// Plan-time ordering of bucket entries (deterministic).
//
// The scatter pass fills every (band, tile, w-base-plane) bucket in an order
// set by atomic cursors.  Here each bucket is re-ordered by a total key: the
// block of rb x cb footprint base cells the entry falls in (rb = cb = 1: the
// base cell itself), then the base cell within the block (row-major, when the
// key has room: neighbouring entries then read the same LDS rows in the
// interpolation, which costs no bank conflicts), then the visibility index,
// which is unique within a bucket.  One 64-bit key per entry, (bucket, block,
// cell, index), is radix-sorted
// with its position (hipCUB, stable); a gather then writes the records and
// weights in that order.  The result depends on the inputs only, so repeated
// plans of the same problem give bitwise-identical gridding.  For the FP32
// w-stacked gridder the gather also writes the w-phase exp(2 pi i s_c w) of
// every entry, evaluated in FP64 and stored FP32.
#include <hipcub/hipcub.hpp>

#include "pfb_kernels.h"

namespace pfb {

namespace {

constexpr int kSortThreads = 256;

int bits_for(uint64_t n) {   // bits to hold values 0 .. n - 1
    int b = 0;
    while (b < 64 && (uint64_t(1) << b) < n) ++b;
    return b;
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void sort_keys_kernel(const Rec<R> *recs, const int64_t *items, int T,
                                                                 int W, int rb, int cb, int sh_cell, int sh_blk,
                                                                 int sh_bucket, uint64_t *keys, uint32_t *vals) {
    const int64_t start = items[4 * blockIdx.x], n = items[4 * blockIdx.x + 1], bucket = items[4 * blockIdx.x + 3];
    const int KS = T + W - 1, NB = (KS + cb - 1) / cb;
    const R hw = R(0.5) * R(W);
    for (int64_t e = threadIdx.x; e < n; e += kSortThreads) {
        const Rec<R> r = recs[start + e];
        const int i0 = (int)dev_floor(r.fu - hw) + 1, j0 = (int)dev_floor(r.fv - hw) + 1;
        const int a = min(max(i0 + W - 1, 0), KS - 1), b = min(max(j0 + W - 1, 0), KS - 1);
        const uint64_t blk = (uint64_t)((a / rb) * NB + b / cb);
        const uint64_t cell = sh_blk > sh_cell ? (uint64_t)((a % rb) * cb + b % cb) : 0;
        keys[start + e] = ((uint64_t)bucket << sh_bucket) | (blk << sh_blk) | (cell << sh_cell) |
                          (uint64_t)(r.idx & ~kHomeBit);
        vals[start + e] = (uint32_t)(start + e);
    }
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void sort_gather_kernel(const Rec<R> *src, const R *src_om, Rec<R> *dst,
                                                                   R *dst_om, const uint32_t *perm, int64_t n,
                                                                   const uint64_t *keys, int sh_bucket,
                                                                   int64_t bucket_per_band, const BandDev *bands,
                                                                   GeomDev geo, cplx<float> *phase) {
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSortThreads) {
        const uint32_t j = perm[i];
        const Rec<R> r = src[j];
        dst[i] = r;
        dst_om[i] = src_om[j];
        if (phase) {
            // exp(2 pi i (w s_c + u l0 + v m0)): the w factor split off the w-stacking and,
            // for a facet centred at pixel offsets (offx, offy), its shift from the phase
            // centre; u l0 = t_u offx / g_x modulo whole turns, t_u = tile row * T + fu
            const int64_t bucket = (int64_t)(keys[i] >> sh_bucket);
            const BandDev bd = bands[bucket / bucket_per_band];
            double t = (bd.w0 + (double)r.fw * bd.dw) * bd.sc;
            if (geo.offx | geo.offy) {
                const int tile = (int)((bucket % bucket_per_band) / geo.nj0max);
                const double tu = (double)(tile / geo.nty) * geo.T + (double)r.fu;
                const double tv = (double)(tile % geo.nty) * geo.T + (double)r.fv;
                t += tu * geo.offx / geo.gx + tv * geo.offy / geo.gy;
            }
            const cplx<double> z = cis_cycles<double>(t - rint(t));
            phase[i] = cplx<float>{(float)z.re, (float)z.im};
        }
    }
}

struct SortScratch {
    size_t keys_in, keys_out, vals_in, vals_out, cub, total;
    size_t cub_bytes;
};

SortScratch scratch_layout(int64_t n) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    SortScratch s{};
    size_t cub_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, cub_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)std::max<int64_t>(n, 1),
                                             0, 64, (hipStream_t)0);
    s.cub_bytes = cub_bytes;
    s.keys_in = 0;
    s.keys_out = s.keys_in + up(n * sizeof(uint64_t));
    s.vals_in = s.keys_out + up(n * sizeof(uint64_t));
    s.vals_out = s.vals_in + up(n * sizeof(uint32_t));
    s.cub = s.vals_out + up(n * sizeof(uint32_t));
    s.total = s.cub + up(cub_bytes);
    return s;
}

}  // namespace

size_t sort_scratch_bytes(int64_t n_entries) { return scratch_layout(n_entries).total; }

int sort_key_bits(int64_t n_buckets, int T, int W, int rb, int cb, int64_t n_vis) {
    const int KS = T + W - 1;
    const int64_t nblk = (int64_t)((KS + rb - 1) / rb) * ((KS + cb - 1) / cb);
    return bits_for((uint64_t)n_buckets) + bits_for((uint64_t)nblk) + bits_for((uint64_t)n_vis);
}

hipError_t launch_sort(bool dbl, const void *src, const void *src_om, void *dst, void *dst_om, const int64_t *items,
                       int n_items, int64_t n_entries, int64_t n_buckets, int64_t bucket_per_band, int64_t n_vis,
                       int T, int W, int rb, int cb, const BandDev *bands, const GeomDev &geo, void *phase,
                       void *scratch, hipStream_t s) {
    if (n_items <= 0 || n_entries <= 0) return hipSuccess;
    const int KS = T + W - 1;
    const int64_t nblk = (int64_t)((KS + rb - 1) / rb) * ((KS + cb - 1) / cb);
    const int sh_cell = bits_for((uint64_t)n_vis);
    int cell_bits = bits_for((uint64_t)rb * cb);
    if (sh_cell + cell_bits + bits_for((uint64_t)nblk) + bits_for((uint64_t)n_buckets) > 64) cell_bits = 0;
    const int sh_blk = sh_cell + cell_bits;
    const int sh_bucket = sh_blk + bits_for((uint64_t)nblk);
    const int end_bit = sh_bucket + bits_for((uint64_t)n_buckets);
    if (end_bit > 64) return hipErrorInvalidValue;
    const SortScratch L = scratch_layout(n_entries);
    char *base = reinterpret_cast<char *>(scratch);
    uint64_t *kin = reinterpret_cast<uint64_t *>(base + L.keys_in);
    uint64_t *kout = reinterpret_cast<uint64_t *>(base + L.keys_out);
    uint32_t *vin = reinterpret_cast<uint32_t *>(base + L.vals_in);
    uint32_t *vout = reinterpret_cast<uint32_t *>(base + L.vals_out);
    if (dbl)
        hipLaunchKernelGGL(sort_keys_kernel<double>, dim3(n_items), dim3(kSortThreads), 0, s,
                           (const Rec<double> *)src, items, T, W, rb, cb, sh_cell, sh_blk, sh_bucket, kin, vin);
    else
        hipLaunchKernelGGL(sort_keys_kernel<float>, dim3(n_items), dim3(kSortThreads), 0, s,
                           (const Rec<float> *)src, items, T, W, rb, cb, sh_cell, sh_blk, sh_bucket, kin, vin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t cub_bytes = L.cub_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(base + L.cub, cub_bytes, kin, kout, vin, vout, (int)n_entries, 0, end_bit, s);
    if (e != hipSuccess) return e;
    const int64_t nb = std::min<int64_t>((n_entries + kSortThreads - 1) / kSortThreads, 65536);
    if (dbl)
        hipLaunchKernelGGL(sort_gather_kernel<double>, dim3(nb), dim3(kSortThreads), 0, s, (const Rec<double> *)src,
                           (const double *)src_om, (Rec<double> *)dst, (double *)dst_om, vout, n_entries, kout,
                           sh_bucket, bucket_per_band, bands, geo, (cplx<float> *)phase);
    else
        hipLaunchKernelGGL(sort_gather_kernel<float>, dim3(nb), dim3(kSortThreads), 0, s, (const Rec<float> *)src,
                           (const float *)src_om, (Rec<float> *)dst, (float *)dst_om, vout, n_entries, kout,
                           sh_bucket, bucket_per_band, bands, geo, (cplx<float> *)phase);
    return hipGetLastError();
}

}  // namespace pfb
