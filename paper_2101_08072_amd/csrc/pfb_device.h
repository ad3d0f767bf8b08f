// Device-side building blocks shared by the gfx950 kernels: complex
// arithmetic, the exponential-of-semicircle (ES) kernel, and LDS-resident
// mixed radix-2/4/8 FFT stages (decimation in time for the row passes, in
// frequency for the split column passes) used by every transform pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfb {

constexpr int kThreads = 256;   // every kernel runs 4 wave64 per workgroup

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R re, im;
};

template <typename R> __device__ __forceinline__ cplx<R> mk(R a, R b) { return cplx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cplx<R> operator*(cplx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R> __device__ __forceinline__ cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV> __device__ __forceinline__ cplx<R> mul_mi(cplx<R> a) {
    return INV ? cplx<R>{-a.im, a.re} : cplx<R>{a.im, -a.re};
}

__device__ __forceinline__ float  dev_exp(float x)  { return expf(x); }
__device__ __forceinline__ double dev_exp(double x) { return exp(x); }
__device__ __forceinline__ float  dev_sqrt(float x)  { return sqrtf(x); }
__device__ __forceinline__ double dev_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float  dev_floor(float x)  { return floorf(x); }
__device__ __forceinline__ double dev_floor(double x) { return floor(x); }
__device__ __forceinline__ void dev_sincospi(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void dev_sincospi(double x, double *s, double *c) { sincospi(x, s, c); }

// exp(2 pi i t) for t in cycles (t already small in magnitude)
template <typename R> __device__ __forceinline__ cplx<R> cis_cycles(R t) {
    R s, c;
    dev_sincospi(R(2) * t, &s, &c);
    return {c, s};
}

// ES kernel phi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)) on |z| < W/2, zero outside
// (Barnett, Magland & af Klinteberg 2019).  inv_hw = 2/W.
template <typename R> __device__ __forceinline__ R es_kernel(R z, R beta, R inv_hw) {
    R t = z * inv_hw;
    R a = R(1) - t * t;
    return a > R(0) ? dev_exp(beta * (dev_sqrt(a) - R(1))) : R(0);
}

// ---------------------------------------------------------------------------
// LDS FFT
// ---------------------------------------------------------------------------
// LDS layout of vectors of length 2^LOG2L for the FFT passes.  Element p of a
// vector sits at pad(p) = p + p / 2^SH + p / 2^(LOG2L-3): the first term
// spreads the butterflies' power-of-two strides over the banks, the second the
// digit-reversed scatter of the input (consecutive inputs land L/8 apart).
// Vectors of a column group are ld elements apart, ld = 1 modulo the elements
// per 128-byte bank row, so that lanes walking across columns hit distinct banks.
template <typename R, int LOG2L> struct Lds {
    static constexpr int L = 1 << LOG2L;
    static constexpr int SH = sizeof(R) == 4 ? 3 : 4;
    static constexpr int HS = LOG2L >= SH + 3 ? LOG2L - 3 : 30;
    static constexpr int EB = 128 / (2 * (int)sizeof(R));
    __host__ __device__ static constexpr int pad(int p) { return p + (p >> SH) + (p >> HS); }
    static constexpr int len = pad(L - 1) + 1;
    static constexpr int ld = len + ((1 - len) % EB + EB) % EB;
};

// Radix plan for L = 2^LOG2L: first stage of radix 2^(LOG2L % 3) (if non-zero), then radix 8.
template <int LOG2L> struct FftPlan {
    static constexpr int L = 1 << LOG2L;
    static constexpr int REM = LOG2L % 3;
    static constexpr int NSTAGE = LOG2L / 3 + (REM ? 1 : 0);
    static __host__ __device__ constexpr int radix(int st) { return (REM && st == 0) ? (1 << REM) : 8; }
};

// Position in LDS of input element n for the in-place DIT sequence (mixed-radix digit reversal).
template <int LOG2L> __device__ __forceinline__ int dit_pos(int n) {
    using P = FftPlan<LOG2L>;
    int pos = 0, M = P::L, x = n;
#pragma unroll
    for (int st = P::NSTAGE - 1; st >= 0; --st) {
        const int R = P::radix(st);
        M /= R;
        pos += (x % R) * M;
        x /= R;
    }
    return pos;
}

template <typename R, bool INV> __device__ __forceinline__ void dft2(cplx<R> *v) {
    cplx<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}
template <typename R, bool INV> __device__ __forceinline__ void dft4(cplx<R> *v) {
    cplx<R> s02 = v[0] + v[2], d02 = v[0] - v[2];
    cplx<R> s13 = v[1] + v[3], d13 = mul_mi<R, INV>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
}
template <typename R, bool INV> __device__ __forceinline__ void dft8(cplx<R> *v) {
    const R h = R(0.70710678118654752440084436210485);
    cplx<R> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<R, INV>(e);
    dft4<R, INV>(o);
    // w8^k for k = 1,2,3 (forward: exp(-2 pi i k / 8))
    cplx<R> o1 = INV ? cplx<R>{h * (o[1].re - o[1].im), h * (o[1].re + o[1].im)}
                     : cplx<R>{h * (o[1].re + o[1].im), h * (o[1].im - o[1].re)};
    cplx<R> o2 = mul_mi<R, INV>(o[2]);
    cplx<R> o3 = INV ? cplx<R>{-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im)}
                     : cplx<R>{h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im)};
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
}
template <typename R, bool INV, int RAD> __device__ __forceinline__ void dft_small(cplx<R> *v) {
    if constexpr (RAD == 2) dft2<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v);
    else dft8<R, INV>(v);
}

// Twiddles exp(-+2 pi i e / Lmax) from a two-level table in LDS: for
// e = e_hi 2^sh + e_lo, w^e = lo[e_lo] hi[e_hi], with lo[k] = w^k (k < 2^sh) and
// hi[k] = w^(k 2^sh) copied from the FP64-accurate forward table in HBM (one
// complex product, about 1.5 ulp; an LDS read instead of a scattered global one).
constexpr int kTwEntries = 256;   // lo + hi entries for Lmax <= 2^14

// The radix-8 stages below the outermost one of an L-point transform
// can take their twiddles from direct tables: for the span m of such a stage
// (the spans are R0 8^s, R0 the radix of the span-1 stage), the values
// w_{8m}^{t j} = exp(-2 pi i t j / (8 m)) for t = 1 .. 7, j < m, at
// off(m) + (t - 1) m + j, copied from the same HBM table and read once each (no
// products, no index arithmetic beyond the butterfly's j).  Whole tables of the smallest spans are kept, as
// many as the kernel's LDS budget allows; mtop is the first span without one.
template <int LOG2L> struct StageTab {
    static constexpr int L = 1 << LOG2L;
    static constexpr int R0 = (LOG2L % 3) ? (1 << (LOG2L % 3)) : 8;
    // entries of the tables of the spans below m
    static __host__ __device__ constexpr int off(int m) {
        int e = 0;
        for (int s = R0; s < m; s *= 8) e += 7 * s;
        return e;
    }
    // entries kept within a budget of maxe
    static __host__ __device__ constexpr int entries(int maxe) {
        int e = 0;
        for (int s = R0; s < L / 8 && e + 7 * s <= maxe; s *= 8) e += 7 * s;
        return e;
    }
    static __host__ __device__ constexpr int mtop(int se) {
        int s = R0;
        for (int e = 0; s < L / 8 && e + 7 * s <= se; s *= 8) e += 7 * s;
        return s;
    }
};
template <typename R> struct TwTab {
    const cplx<R> *lo, *hi;
    int sh, mask;
    const cplx<R> *st;   // direct tables of the spans below mtop
    int mtop;
    __device__ __forceinline__ cplx<R> get(int e) const { return lo[e & mask] * hi[e >> sh]; }
};
// fill the two-level table at lds (kTwEntries elements) from the table of length
// 2^log2_lmax, and after it the SE entries of the direct tables of a 2^LOG2L-point
// transform (SE = StageTab<LOG2L>::entries(budget)); the caller synchronises the
// block before the first use
template <typename R, int NT, int LOG2L, int SE>
__device__ __forceinline__ TwTab<R> tw_fill(cplx<R> *lds, const cplx<R> *tw, int log2_lmax) {
    using ST = StageTab<LOG2L>;
    const int sh = (log2_lmax + 1) / 2, nlo = 1 << sh, nhi = 1 << (log2_lmax - sh);
    for (int k = threadIdx.x; k < nlo + nhi; k += NT) lds[k] = k < nlo ? tw[k] : tw[(k - nlo) << sh];
    cplx<R> *st = lds + kTwEntries;
    for (int k = threadIdx.x; k < SE; k += NT) {
        int m = ST::R0, o = 0;
        while (k >= o + 7 * m) {
            o += 7 * m;
            m *= 8;
        }
        const int t = (k - o) / m + 1, j = k - o - (t - 1) * m;
        st[k] = tw[(t * j * (ST::L / (8 * m))) << (log2_lmax - LOG2L)];
    }
    return TwTab<R>{lds, lds + nlo, sh, nlo - 1, st, ST::mtop(SE)};
}
template <typename R, bool INV> __device__ __forceinline__ cplx<R> twiddle(const TwTab<R> &tt, int e) {
    cplx<R> w = tt.get(e);
    return INV ? conj(w) : w;
}

// v[t] *= w^(t j) for t = 1 .. 7 from a direct table (p = st + off(m) + j)
template <typename R, bool INV> __device__ __forceinline__ void stage_twiddles_tab(cplx<R> *v, const cplx<R> *p, int m) {
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        const cplx<R> w = p[(t - 1) * m];
        v[t] = v[t] * (INV ? conj(w) : w);
    }
}

// v[t] *= w^(t e) for t = 1 .. RAD - 1
template <typename R, bool INV, int RAD>
__device__ __forceinline__ void stage_twiddles(cplx<R> *v, const TwTab<R> &tw, int e) {
    if constexpr (RAD == 8) {
        // three table reads; w^3, w^5, w^6, w^7 as products (a few ulp)
        const cplx<R> w1 = twiddle<R, INV>(tw, e), w2 = twiddle<R, INV>(tw, 2 * e), w4 = twiddle<R, INV>(tw, 4 * e);
        const cplx<R> w3 = w1 * w2;
        v[1] = v[1] * w1;
        v[2] = v[2] * w2;
        v[3] = v[3] * w3;
        v[4] = v[4] * w4;
        v[5] = v[5] * (w1 * w4);
        v[6] = v[6] * (w2 * w4);
        v[7] = v[7] * (w3 * w4);
    } else {
#pragma unroll
        for (int t = 1; t < RAD; ++t) v[t] = v[t] * twiddle<R, INV>(tw, t * e);
    }
}

// One DIT stage of radix RAD at span m over C vectors stored at buf + c*ld.
template <typename R, bool INV, int RAD, int LOG2L, int NT>
__device__ __forceinline__ void dit_stage(cplx<R> *buf, int C, int ld, int m, const TwTab<R> &tw, int tw_shift) {
    constexpr int L = 1 << LOG2L;
    constexpr int NB = L / RAD;               // butterflies per vector
    const int total = NB * C;
    // table index step for w_{RAD m}^{t j}: Lmax / (RAD m) = (Lmax / L) * (L / (RAD m))
    const int estep = (L / (RAD * m)) << tw_shift;
    for (int id = threadIdx.x; id < total; id += NT) {
        const int c = id / NB;
        const int bfly = id - c * NB;
        const int j = bfly % m;
        const int g = bfly / m;
        const int base = g * RAD * m + j;
        // base = g RAD m + j (j < m) and t m (t < RAD) occupy disjoint bits, so the
        // sum never carries and pad(base + t m) = pad(base) + pad(t m): one
        // address per butterfly plus constant offsets once the stage is unrolled
        cplx<R> *vb = buf + c * ld + Lds<R, LOG2L>::pad(base);
        cplx<R> v[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) v[t] = vb[Lds<R, LOG2L>::pad(t * m)];
        if (RAD == 8 && m > 1 && m < tw.mtop) stage_twiddles_tab<R, INV>(v, tw.st + StageTab<LOG2L>::off(m) + j, m);
        else if (m > 1) stage_twiddles<R, INV, RAD>(v, tw, j * estep);
        dft_small<R, INV, RAD>(v);
#pragma unroll
        for (int t = 0; t < RAD; ++t) vb[Lds<R, LOG2L>::pad(t * m)] = v[t];
    }
}

// Full in-place FFT of C vectors of length 2^LOG2L already loaded in DIT order,
// by a block of NT threads.  Ends with a barrier; the result is in natural
// order at Lds<R, LOG2L>::pad(k).
template <typename R, bool INV, int LOG2L, int NT = kThreads>
__device__ __forceinline__ void lds_fft(cplx<R> *buf, int C, int ld, const TwTab<R> &tw, int tw_shift) {
    using P = FftPlan<LOG2L>;
    int m = 1;
#pragma unroll
    for (int st = 0; st < P::NSTAGE; ++st) {
        constexpr int dummy = 0;
        (void)dummy;
        const int RAD = P::radix(st);
        if (RAD == 2) dit_stage<R, INV, 2, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        else if (RAD == 4) dit_stage<R, INV, 4, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        else dit_stage<R, INV, 8, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        m *= RAD;
        __syncthreads();
    }
}

// One decimation-in-frequency stage: the transpose of dit_stage (the radix-RAD
// DFT first, then the twiddles of the same butterfly).
template <typename R, bool INV, int RAD, int LOG2L, int NT>
__device__ __forceinline__ void dif_stage(cplx<R> *buf, int C, int ld, int m, const TwTab<R> &tw, int tw_shift) {
    constexpr int L = 1 << LOG2L;
    constexpr int NB = L / RAD;
    const int total = NB * C;
    const int estep = (L / (RAD * m)) << tw_shift;
    for (int id = threadIdx.x; id < total; id += NT) {
        const int c = id / NB;
        const int bfly = id - c * NB;
        const int j = bfly % m;
        const int g = bfly / m;
        cplx<R> *vb = buf + c * ld + Lds<R, LOG2L>::pad(g * RAD * m + j);
        cplx<R> v[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) v[t] = vb[Lds<R, LOG2L>::pad(t * m)];
        dft_small<R, INV, RAD>(v);
        if (RAD == 8 && m > 1 && m < tw.mtop) stage_twiddles_tab<R, INV>(v, tw.st + StageTab<LOG2L>::off(m) + j, m);
        else if (m > 1) stage_twiddles<R, INV, RAD>(v, tw, j * estep);
#pragma unroll
        for (int t = 0; t < RAD; ++t) vb[Lds<R, LOG2L>::pad(t * m)] = v[t];
    }
}

// In-place FFT of C vectors given in natural order at Lds::pad(n); the result
// X[k] is left at Lds::pad(dit_pos<LOG2L>(k)), which is the input order of
// lds_fft.  The DFT matrix is symmetric, so the transpose of lds_fft's sequence
// (stages in reverse order, each transposed) computes it.  Ends with a barrier.
template <typename R, bool INV, int LOG2L, int NT = kThreads>
__device__ __forceinline__ void lds_fft_dif(cplx<R> *buf, int C, int ld, const TwTab<R> &tw, int tw_shift) {
    using P = FftPlan<LOG2L>;
    int m = P::L;
#pragma unroll
    for (int st = P::NSTAGE - 1; st >= 0; --st) {
        const int RAD = P::radix(st);
        m /= RAD;   // span of DIT stage st: the product of the radices before it
        if (RAD == 2) dif_stage<R, INV, 2, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        else if (RAD == 4) dif_stage<R, INV, 4, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        else dif_stage<R, INV, 8, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        __syncthreads();
    }
}

// Inverse of dit_pos: the input index n whose DIT position is q.
template <int LOG2L> __device__ __forceinline__ int dit_inv(int q) {
    using P = FftPlan<LOG2L>;
    int n = 0, W = P::L, x = q;
#pragma unroll
    for (int st = 0; st < P::NSTAGE; ++st) {
        const int R = P::radix(st);
        W /= R;   // weight of this digit in n: the product of the later stages' radices
        n += (x % R) * W;
        x /= R;
    }
    return n;
}

// base-8 digit reversal of q over D digits
template <int D> __device__ __forceinline__ int rev8(int q) {
    int r = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        r = (r << 3) | (q & 7);
        q >>= 3;
    }
    return r;
}

// Input and output of the row transforms go in two steps each, so that all the
// global loads of a thread's batch are issued before any of them is waited for
// (a load whose value is used at once, or a store between loads, would expose
// each load's latency in turn):
//   fetch_in(c, r)          loads of input r of vector c (no arithmetic, no stores)
//   make_in(c, r, raw)      the input value from them (arithmetic, side effects)
//   fetch_out(c, k)         loads that output k of vector c needs
//   put_out(c, k, v, raw)   its stores
struct NoRaw {};
struct InPlain {   // make_in for inputs loaded as they are
    template <class T> __device__ __forceinline__ T operator()(int, int, const T &raw) const { return raw; }
};
struct OutNoFetch {
    __device__ __forceinline__ NoRaw operator()(int, int) const { return NoRaw{}; }
};
// items per thread whose loads are in flight together in the unfused input and
// output loops: eight, or four in 1024-thread blocks (two of them per CU leave 64
// registers per lane); a caller may ask for another input batch (UIN)
template <class Raw, int NT> constexpr int io_batch() { return NT >= 1024 ? 4 : 8; }

// FFT of C vectors of length 2^LOG2L (2^5 .. 2^14) whose first stage reads its
// inputs through fetch_in / make_in (natural order n) and, with STORE_REGS, whose
// last stage hands its outputs to fetch_out / put_out (natural order k) instead
// of writing them to LDS; without STORE_REGS the result is in LDS at
// Lds::pad(k) after a final barrier.  The first stage (radix R0, span 1) takes
// inputs t Q + q (Q = L / R0, t < R0): its outputs belong at DIT positions
// rev8(q) R0 + t, which replaces the digit-reversed scatter and one LDS pass.
template <typename R, bool INV, int LOG2L, int NT, bool STORE_REGS, class FIn, class MIn, class FOut, class POut>
__device__ __forceinline__ void lds_fft_io(cplx<R> *buf, int C, int ld, const TwTab<R> &tw, int tw_shift,
                                           FIn fetch_in, MIn make_in, FOut fetch_out, POut put_out) {
    using P = FftPlan<LOG2L>;
    constexpr int L = 1 << LOG2L;
    constexpr int S = P::NSTAGE;
    constexpr int R0 = P::radix(0);
    constexpr int Q = L / R0;
    static_assert(S >= 2, "at least two stages");
    using Raw = decltype(fetch_in(0, 0));
    // G = 8 / R0 butterflies per thread and iteration keep eight loads in flight;
    // when the thread count divides the work no bounds test separates the loads
    constexpr int G = 8 / R0;
    constexpr bool EXACT = Q % (G * NT) == 0;
    for (int id0 = threadIdx.x; id0 < C * Q; id0 += G * NT) {
        Raw raw[G][R0];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int id = id0 + u * NT;
            if (EXACT || id < C * Q) {
                const int c = id / Q, q = id - c * Q;
#pragma unroll
                for (int t = 0; t < R0; ++t) raw[u][t] = fetch_in(c, t * Q + q);
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int id = id0 + u * NT;
            if (EXACT || id < C * Q) {
                const int c = id / Q, q = id - c * Q;
                cplx<R> v[R0];
#pragma unroll
                for (int t = 0; t < R0; ++t) v[t] = make_in(c, t * Q + q, raw[u][t]);
                dft_small<R, INV, R0>(v);
                cplx<R> *vb = buf + c * ld + Lds<R, LOG2L>::pad(rev8<S - 1>(q) * R0);
#pragma unroll
                for (int t = 0; t < R0; ++t) vb[Lds<R, LOG2L>::pad(t)] = v[t];
            }
        }
    }
    __syncthreads();
    int m = R0;
    constexpr int LAST = STORE_REGS ? S - 1 : S;
#pragma unroll
    for (int st = 1; st < LAST; ++st) {
        dit_stage<R, INV, 8, LOG2L, NT>(buf, C, ld, m, tw, tw_shift);
        m *= 8;
        __syncthreads();
    }
    if constexpr (STORE_REGS) {
        // last stage: span m = L / 8; butterfly j holds outputs j + t m
        constexpr int M = L / 8;
        using ORaw = decltype(fetch_out(0, 0));
        for (int id = threadIdx.x; id < C * M; id += NT) {
            const int c = id / M, j = id - c * M;
            ORaw oraw[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) oraw[t] = fetch_out(c, j + t * M);
            const cplx<R> *vb = buf + c * ld + Lds<R, LOG2L>::pad(j);
            cplx<R> v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = vb[Lds<R, LOG2L>::pad(t * M)];
            stage_twiddles<R, INV, 8>(v, tw, j << tw_shift);
            dft_small<R, INV, 8>(v);
#pragma unroll
            for (int t = 0; t < 8; ++t) put_out(c, j + t * M, v[t], oraw[t]);
        }
    }
}

// lds_fft_io when FUSE, else the same interface over the plain sequence: every
// input scattered to its DIT position, lds_fft, and (STORE_REGS) every output
// read back from LDS.  The fused first stage measured slower where it starts with
// radix 2 or 4.
template <typename R, bool INV, int LOG2L, int NT, bool STORE_REGS, bool FUSE, int UIN = 0, class FIn, class MIn,
          class FOut, class POut>
__device__ __forceinline__ void row_fft(cplx<R> *buf, int C, int ld, const TwTab<R> &tw, int tw_shift, FIn fetch_in,
                                        MIn make_in, FOut fetch_out, POut put_out) {
    if constexpr (FUSE) {
        lds_fft_io<R, INV, LOG2L, NT, STORE_REGS>(buf, C, ld, tw, tw_shift, fetch_in, make_in, fetch_out, put_out);
    } else {
        constexpr int L = 1 << LOG2L;
        using Raw = decltype(fetch_in(0, 0));
        constexpr int U = UIN ? UIN : io_batch<Raw, NT>();
        constexpr bool EXACT = L % (U * NT) == 0;
        for (int id0 = threadIdx.x; id0 < C * L; id0 += U * NT) {
            Raw raw[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int id = id0 + u * NT;
                if (EXACT || id < C * L) {
                    const int c = id / L, r = id - c * L;
                    raw[u] = fetch_in(c, r);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int id = id0 + u * NT;
                if (EXACT || id < C * L) {
                    const int c = id / L, r = id - c * L;
                    buf[c * ld + Lds<R, LOG2L>::pad(dit_pos<LOG2L>(r))] = make_in(c, r, raw[u]);
                }
            }
        }
        __syncthreads();
        lds_fft<R, INV, LOG2L, NT>(buf, C, ld, tw, tw_shift);
        if constexpr (STORE_REGS) {
            using ORaw = decltype(fetch_out(0, 0));
            constexpr int UO = io_batch<ORaw, NT>();
            constexpr bool EXO = L % (UO * NT) == 0;
            for (int id0 = threadIdx.x; id0 < C * L; id0 += UO * NT) {
                ORaw oraw[UO];
#pragma unroll
                for (int u = 0; u < UO; ++u) {
                    const int id = id0 + u * NT;
                    if (EXO || id < C * L) {
                        const int c = id / L, k = id - c * L;
                        oraw[u] = fetch_out(c, k);
                    }
                }
#pragma unroll
                for (int u = 0; u < UO; ++u) {
                    const int id = id0 + u * NT;
                    if (EXO || id < C * L) {
                        const int c = id / L, k = id - c * L;
                        put_out(c, k, buf[c * ld + Lds<R, LOG2L>::pad(k)], oraw[u]);
                    }
                }
            }
        }
    }
}
// the fused form for lengths whose plan starts with radix 8
template <int LOG2L> constexpr bool fuse_first8() { return FftPlan<LOG2L>::REM == 0; }

}  // namespace pfb
